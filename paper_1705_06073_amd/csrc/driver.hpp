// a9: the estimator's block-coordinate descent (Sec. II-C/E) as a resumable
// per-instance state machine.  One call consumes the results of the last
// evaluation round (C at the requested point: ln|C|, y^H C^{-1} y, ||w||^2,
// the active vectors q..x, and the FP64 q, s at grid candidates) and runs the
// algorithm until it needs the next evaluation, which it requests by writing
// the evaluation point and request bits; or it finishes and writes outputs.
//
// Plain C++ templated on a team: the lanes that run one instance together.
// Every lane of a team runs the same scalar logic on the same values, loops
// over the instance's vectors are strided over the lanes, and team reductions
// return the same bits in every lane, so all lanes take the same branches.
// The device kernel uses one wave as the team; the host build one thread.
#pragma once
#include <math.h>
#include <stdint.h>

#ifndef SFLS_HD
#define SFLS_HD __host__ __device__
#endif

namespace sfls {

struct DrvParams {
  double tau, tol_obj, tol_newton, eps_beta_rel, eps_L, approx_ratio, approx_min_dist, ls_c1,
      curv_eps, polish_tol, polish_ftol;
  int32_t J, max_inner, max_outer, approx_max_iters, approx_use_tau, ls_max, polish_max_iters,
      cand_cap;
};

// phases
enum : int32_t {
  PH_START = 0,
  PH_APPROX_WAIT,
  PH_EXACT_WAIT,
  PH_BETA_WAIT,
  PH_INNER_WAIT,
  PH_LS_WAIT,
  PH_DEACT_WAIT,
  PH_TERM_WAIT,
  PH_POLISH_WAIT,
  PH_DONE
};

// Scalar state of one instance.
struct DrvState {
  int32_t phase, it, inner, pit, ls_trial, K, approx_on, z_changed, cur_valid, converged,
      cap_hit, polish, mem_n, mem_head, kstar, status, nevals, done, saved, pad_;
  double beta, zeta, eps_beta, yy, L_prev, f_cur, lam2, alpha, amax, gd, nu0;
};

// Per-instance array views (device pointers, offset to this instance).
struct DrvArrays {
  int N, L, kcap;
  // observations per vector (Sec. II-A; N for complete data): the count
  // scales of Sec. II-E (initial beta, eps_beta, the stopping rules,
  // K_max = M in the prior and eq. zetaUpdate) are in M, the frequency
  // scales (grid, distances, the refinement's tolerance) in N
  int Mo = 0;
  // observation vectors (Sec. V): the per-vector arrays ev_q, ev_r, ev_u,
  // q_save, cand_q and out_alpha hold vector g at g * (vk, vk, vk, vk, vc, vo)
  // doubles from the instance's entry (G = 1: the single-vector model)
  int G = 1;
  int64_t vk = 0, vc = 0, vo = 0;
  // current accepted point
  double* th;
  double* ga;
  // evaluation point (read by the evaluation kernels)
  double* th_e;
  double* ga_e;
  int32_t* K_e;     // number of components at the evaluation point
  double* beta_e;   // beta at the evaluation point
  int32_t* req;     // request bits for the next round
  double* gbar_e;   // gamma_bar for the grid stage (<= 0: per-point optimum)
  double* zeta_e;   // zeta for the grid stage
  // L-BFGS storage
  double* g;        // gradient at the current point [2 kcap]
  double* d;        // direction [2 kcap]
  double* Sm;       // [J][2 kcap]
  double* Ym;       // [J][2 kcap]
  double* rhom;     // [J]
  double* am;       // [J] two-loop scratch
  double* gt;       // gradient at the trial [2 kcap]
  double* q_save;   // q at the polish's current point (complex) [2 kcap]
  // evaluation results (written by the kernels, valid for the last request)
  double* ev_q;  // complex [kcap] interleaved
  double* ev_r;
  double* ev_u;
  double* ev_s;
  double* ev_t;
  double* ev_v;
  double* ev_x;
  double* logdet;
  double* yCy;
  double* ww;
  const int32_t* lev_status;
  const int32_t* cand;    // grid indices, cand[0] = argmin
  const int32_t* ncand;
  const double* cand_q;   // complex
  const double* cand_s;
  // approximate-scheme scratch [cand_cap + 1]
  double* cbuf_dl;
  double* cbuf_gh;
  int32_t* cbuf_l;
  // outputs
  int64_t* out_K;
  double* out_theta;
  double* out_alpha;  // complex
  double* out_gamma;
  double* out_beta;
  double* out_zeta;
  double* out_obj;
  int32_t* out_iters;
  int32_t* out_evals;
  int32_t* out_status;
  // Shadow evaluation slot (speculative line-search trials; all NULL when
  // off).  A rejected trial of a line search (inner or final refinement) is
  // followed by the trial at half its step; when a trial is requested the driver also writes that
  // next point into the shadow slot and sets *sh_wish, and the round's grant
  // (one workgroup) turns wishes into shadow requests while CUs are free.  A
  // granted shadow (*sh_req set) was evaluated in the same round as the
  // trial, so a rejection continues with it at once instead of a round later;
  // the points evaluated and the arithmetic are those without the shadow.
  double* sh_th_e = nullptr;
  double* sh_ga_e = nullptr;
  int32_t* sh_K_e = nullptr;
  double* sh_beta_e = nullptr;
  double* sh_gbar_e = nullptr;
  double* sh_zeta_e = nullptr;
  const int32_t* sh_req = nullptr;
  int32_t* sh_wish = nullptr;
  const double* sh_ev_q = nullptr;  // complex [kcap] interleaved, as ev_q
  const double* sh_ev_r = nullptr;
  const double* sh_ev_u = nullptr;
  const double* sh_ev_s = nullptr;
  const double* sh_ev_t = nullptr;
  const double* sh_ev_v = nullptr;
  const double* sh_ev_x = nullptr;
  const double* sh_logdet = nullptr;
  const double* sh_yCy = nullptr;
  const double* sh_ww = nullptr;
  const int32_t* sh_lev_status = nullptr;
};

SFLS_HD inline double xlogy_(double a, double b) { return a == 0.0 ? 0.0 : a * log(b); }
SFLS_HD inline double prior_term(int K, int N, double z) {
  return -(xlogy_((double)K, z) + xlogy_((double)(N - K), 1.0 - z));
}
SFLS_HD inline double wrapd(double a, double b) {
  double d = fabs(a - b);
  d = d - floor(d);
  return fmin(d, 1.0 - d);
}
// The single-component quantities of Sec. II-D (eqs. activate_gamma, delta_L,
// activate_criterion) and, for G observation vectors, of eq. singlecomp-mmv,
// with q2 = sum_g |q_g|^2:
//   gamma_hat = (q2/G - s)/s^2,  Delta L = G ln(1 + gb s) + ln((1-zeta)/zeta)
//   - q2/(1/gb + s), and the criterion q2/(G s) > (1 + 1/(gb s)) (ln(1 + gb s)
//   + ln((1-zeta)/zeta)/G) + tau (the single-vector form on the per-vector
//   average).  Written so that G = 1 performs the single-vector operations.
SFLS_HD inline double gamma_hat(double q2, double s, int G = 1) {
  const double qb = G == 1 ? q2 : q2 / (double)G;
  return (qb / s > 1.0) ? (qb - s) / (s * s) : 0.0;
}
SFLS_HD inline double delta_L(double q2, double s, double gb, double zeta, int G = 1) {
  double lg = log((1.0 + gb * s) * ((1.0 - zeta) / zeta));
  if (G != 1) lg += (double)(G - 1) * log1p(gb * s);
  return lg - ((gb > 0.0) ? q2 / (1.0 / gb + s) : 0.0);
}
SFLS_HD inline bool act_criterion(double q2, double s, double gb, double zeta, double tau,
                                  int G = 1) {
  const double kap = (G == 1 ? q2 : q2 / (double)G) / s;
  double lg = log((1.0 + gb * s) * ((1.0 - zeta) / zeta));
  if (G != 1) lg = (lg + (double)(G - 1) * log1p(gb * s)) / (double)G;
  const double rhs = (1.0 + 1.0 / (gb * s)) * lg + tau;
  if (rhs != rhs) return false;
  return kap > rhs;
}

// One thread as the team (host build).
struct SerialTeam {
  SFLS_HD static int lane() { return 0; }
  SFLS_HD static int width() { return 1; }
  SFLS_HD static double sum(double v) { return v; }
  SFLS_HD static double max(double v) { return v; }
  SFLS_HD static double min(double v) { return v; }
  SFLS_HD static int imin(int v) { return v; }
  SFLS_HD static bool any(bool b) { return b; }
  SFLS_HD static void sync() {}
};

template <typename T>
struct Driver {
  const DrvParams& P;
  DrvState& S;
  const DrvArrays& A;
  int N, J;

  int Mo;

  SFLS_HD Driver(const DrvParams& p, DrvState& s, const DrvArrays& a)
      : P(p), S(s), A(a), N(a.N), J(p.J), Mo(a.Mo > 0 ? a.Mo : a.N) {}

  // L_MMV = G ln|C| + sum_g y_g^H C^{-1} y_g - prior (Sec. V; G = 1: eq. obj)
  SFLS_HD double f_of_eval() const {
    const double ld = A.G == 1 ? *A.logdet : (double)A.G * *A.logdet;
    return ld + *A.yCy + prior_term(S.K, Mo, S.zeta);
  }

  // the scale of the stopping rules: M, or G M for G observation vectors (the
  // objective is a sum of G single-vector objectives)
  SFLS_HD double gN() const { return A.G == 1 ? (double)Mo : (double)A.G * (double)Mo; }

  SFLS_HD double gbar() const {
    if (S.K == 0) return -1.0;
    double s = 0.0;
    for (int k = T::lane(); k < S.K; k += T::width()) s += A.ga[k];
    return T::sum(s) / (double)S.K;
  }

  // request an evaluation at the current point (th, ga, beta).  When the
  // last evaluation is already at that point (cur_valid), its factor, C^{-1}y
  // and active vectors are still in place and only the grid stage runs.
  SFLS_HD void request_current(int32_t bits) {
    if (S.cur_valid) bits &= ~1;  // REQ_EVAL
    for (int k = T::lane(); k < S.K; k += T::width()) { A.th_e[k] = A.th[k]; A.ga_e[k] = A.ga[k]; }
    *A.K_e = S.K;
    *A.beta_e = S.beta;
    *A.gbar_e = gbar();
    *A.zeta_e = S.zeta;
    *A.req = bits;
    if (bits & 1) S.nevals += 1;
  }

  // gradient and replaced diagonal Hessian of component k from the
  // evaluation results (eqs. derivative, derivative2; replacements (50N)^2
  // and gamma^-2)
  // (with G observation vectors the sums over g of the single-vector
  // expressions, Sec. V: q, r, u per vector, s, t, v, x shared)
  SFLS_HD void deriv_k(int k, double gk, double& gth, double& gga, double& hth,
                       double& hga) const {
    const double s = A.ev_s[2 * k];
    const double tr = A.ev_t[2 * k], ti = A.ev_t[2 * k + 1];
    const double vr = A.ev_v[2 * k];
    const double xr = A.ev_x[2 * k];
    const double t2r = tr * tr - ti * ti;
    const double xsr = xr * s;
    double im_sum = 0.0, gga_sum = 0.0, inner = 0.0, hga_sum = 0.0;
    for (int gv = 0; gv < A.G; ++gv) {
      const int64_t o = gv * A.vk;
      const double qr = A.ev_q[o + 2 * k], qi = A.ev_q[o + 2 * k + 1];
      const double rr = A.ev_r[o + 2 * k], ri = A.ev_r[o + 2 * k + 1];
      const double ur = A.ev_u[o + 2 * k], ui = A.ev_u[o + 2 * k + 1];
      const double q2 = qr * qr + qi * qi, r2 = rr * rr + ri * ri;
      // Im(t - conj(q) r)
      const double im_t_qr = ti - (qr * ri - qi * rr);
      // Re{ x - v + g(t^2 - x s) + g(x|q|^2 + s|r|^2 - 2 t r conj q) + (u conj q - |r|^2) }
      // t r conj(q)
      const double trr = tr * rr - ti * ri, tri = tr * ri + ti * rr;
      const double trq = trr * qr + tri * qi;
      const double uq = ur * qr + ui * qi;
      const double in_g = xr - vr + gk * (t2r - xsr) + gk * (xr * q2 + s * r2 - 2.0 * trq) +
                          (uq - r2);
      const double hga_g = 2.0 * s * q2 - s * s;
      if (gv == 0) {
        im_sum = im_t_qr; gga_sum = s - q2; inner = in_g; hga_sum = hga_g;
      } else {
        im_sum += im_t_qr; gga_sum += s - q2; inner += in_g; hga_sum += hga_g;
      }
    }
    gth = 2.0 * gk * im_sum;
    gga = gga_sum;
    hth = 2.0 * gk * inner;
    hga = hga_sum;
    if (!(hth > 0.0)) hth = (50.0 * N) * (50.0 * N);
    if (!(hga > 0.0)) hga = (gk > 0.0) ? 1.0 / (gk * gk) : 1.0;
  }

  // gradient g and (if h) replaced diagonal Hessian at the evaluated point
  SFLS_HD void derivs(const double* __restrict__ gam, double* __restrict__ g,
                      double* __restrict__ h) const {
    const int K = S.K;
    for (int k = T::lane(); k < K; k += T::width()) {
      double gth, gga, hth, hga;
      deriv_k(k, gam[k], gth, gga, hth, hga);
      g[k] = gth;
      g[K + k] = gga;
      if (h) {
        h[k] = hth;
        h[K + k] = hga;
      }
    }
    T::sync();
  }

  // diagonal Newton decrement sum_i g_i^2 / h_i at the evaluated point
  SFLS_HD double newton_dec(const double* __restrict__ gam) const {
    double nu = 0.0;
    for (int k = T::lane(); k < S.K; k += T::width()) {
      double gth, gga, hth, hga;
      deriv_k(k, gam[k], gth, gga, hth, hga);
      nu += gth * gth / hth + gga * gga / hga;
    }
    return T::sum(nu);
  }

  SFLS_HD double dot(const double* __restrict__ a, const double* __restrict__ b, int n) const {
    double s = 0.0;
    for (int i = T::lane(); i < n; i += T::width()) s += a[i] * b[i];
    return T::sum(s);
  }
  // d += a * x
  SFLS_HD static void axpy(double a, const double* __restrict__ x, double* __restrict__ d, int n) {
    for (int e = T::lane(); e < n; e += T::width()) d[e] += a * x[e];
  }

  SFLS_HD void mem_reset() { S.mem_n = 0; S.mem_head = 0; }

  SFLS_HD double* mem_s(int i) const { return A.Sm + (int64_t)i * 2 * A.kcap; }
  SFLS_HD double* mem_y(int i) const { return A.Ym + (int64_t)i * 2 * A.kcap; }

  // slot of the i-th oldest pair
  SFLS_HD int mem_slot(int i) const { return (S.mem_head - S.mem_n + i + J) % J; }

  SFLS_HD void mem_push(const double* s, const double* y, int n) {
    double sy = dot(s, y, n), ss = dot(s, s, n), yy = dot(y, y, n);
    if (!(sy > P.curv_eps * sqrt(ss) * sqrt(yy))) return;
    const int slot = S.mem_head;
    double* __restrict__ ds = mem_s(slot);
    double* __restrict__ dy = mem_y(slot);
    for (int i = T::lane(); i < n; i += T::width()) { ds[i] = s[i]; dy[i] = y[i]; }
    A.rhom[slot] = 1.0 / sy;
    S.mem_head = (S.mem_head + 1) % J;
    if (S.mem_n < J) S.mem_n += 1;
  }

  // two-loop recursion with H0 = diag(1/h); d = -H g.  Falls back to -g/h
  // (after a reset) when the result is not a descent direction.
  SFLS_HD void direction(const double* __restrict__ g, const double* __restrict__ h,
                         double* __restrict__ d, int n) {
    for (int i = T::lane(); i < n; i += T::width()) d[i] = g[i];
    for (int i = S.mem_n - 1; i >= 0; --i) {
      const int sl = mem_slot(i);
      const double a = A.rhom[sl] * dot(mem_s(sl), d, n);
      A.am[sl] = a;
      axpy(-a, mem_y(sl), d, n);
    }
    for (int e = T::lane(); e < n; e += T::width()) d[e] /= h[e];
    for (int i = 0; i < S.mem_n; ++i) {
      const int sl = mem_slot(i);
      const double bta = A.rhom[sl] * dot(mem_y(sl), d, n);
      axpy(A.am[sl] - bta, mem_s(sl), d, n);
    }
    bool bad = false;
    double gd = 0.0;
    for (int e = T::lane(); e < n; e += T::width()) {
      const double de = -d[e];
      d[e] = de;
      if (!(de == de) || isinf(de)) bad = true;
      gd += g[e] * de;
    }
    const bool ok = !T::any(bad);
    gd = T::sum(gd);
    if (!ok || gd >= 0.0) {
      mem_reset();
      for (int e = T::lane(); e < n; e += T::width()) d[e] = -g[e] / h[e];
    }
    T::sync();
  }

  // set up a line search from the current point along d
  SFLS_HD void ls_begin(bool polish) {
    const int K = S.K;
    const double* d = A.d;
    S.gd = dot(A.g, d, 2 * K);
    // largest step keeping every gamma >= 0, and the first k reaching it
    double amax = INFINITY;
    int kstar = -1;
    for (int k = T::lane(); k < K; k += T::width()) {
      const double dg = d[K + k];
      if (dg < 0.0) {
        const double r = A.ga[k] / (-dg);
        if (r < amax) { amax = r; kstar = k; }
      }
    }
    const double am = T::min(amax);
    kstar = T::imin((kstar >= 0 && amax == am) ? kstar : INT32_MAX);
    S.amax = am;
    S.kstar = kstar == INT32_MAX ? -1 : kstar;
    // the first trial from the team's limit (every lane steps by the same alpha)
    if (polish) S.alpha = (am > 1.0) ? 1.0 : 0.5 * am;
    else S.alpha = fmin(1.0, am);
    S.ls_trial = 0;
    S.polish = polish ? 1 : 0;
  }

  // the trial point at step alpha (as the evaluation kernels read it)
  SFLS_HD void trial_point(double alpha, double* th_e, double* ga_e) const {
    const int K = S.K;
    // the component that limits a full step lands on gamma = 0 exactly
    const int kz = (!S.polish && alpha == S.amax) ? S.kstar : -1;
    for (int k = T::lane(); k < K; k += T::width()) {
      double t = A.th[k] + alpha * A.d[k];
      t = t - floor(t);
      if (t >= 1.0) t = 0.0;
      th_e[k] = t;
      double gk = A.ga[k] + alpha * A.d[K + k];
      ga_e[k] = (k == kz) ? 0.0 : (gk > 0.0 ? gk : 0.0);
    }
  }

  // whether a rejection of the trial at alpha ends the search (the tests of
  // L_LS_RESULT at the halved step); dmax = max |d_theta| (polish only)
  SFLS_HD bool gives_up_after(double alpha, double dmax) const {
    if (S.ls_trial + 1 >= P.ls_max) return true;
    const double ah = alpha * 0.5;
    if (S.polish) return ah * dmax < P.polish_tol / (double)N;
    return P.ls_c1 * ah * fabs(S.gd) < P.polish_ftol * (1.0 + fabs(S.f_cur));
  }

  SFLS_HD void ls_request() {
    const int K = S.K;
    trial_point(S.alpha, A.th_e, A.ga_e);
    *A.K_e = K;
    *A.beta_e = S.beta;
    const double gb = gbar();
    *A.gbar_e = gb;
    *A.zeta_e = S.zeta;
    *A.req = 1;  // REQ_EVAL
    S.nevals += 1;
    S.cur_valid = 0;
    // the search's next trial, should this one be rejected
    if (A.sh_wish) {
      double dm = 0.0;  // max |d_theta|, read by the refinement's test only
      if (S.polish) {
        for (int k = T::lane(); k < K; k += T::width()) dm = fmax(dm, fabs(A.d[k]));
        dm = T::max(dm);
      }
      if (!gives_up_after(S.alpha, dm)) {
        trial_point(S.alpha * 0.5, A.sh_th_e, A.sh_ga_e);
        T::sync();
        if (T::lane() == 0) {
          *A.sh_K_e = K;
          *A.sh_beta_e = S.beta;
          *A.sh_gbar_e = gb;
          *A.sh_zeta_e = S.zeta;
          *A.sh_wish = 1;
        }
      }
    }
  }

  // Continue with the shadow evaluation of the halved trial, which the
  // rejected trial's search requests next: its point and results become the
  // trial's, as if it had been requested and evaluated now.
  SFLS_HD bool take_shadow() {
    if (!A.sh_req || !(*A.sh_req & 1) || *A.sh_lev_status != 0) return false;
    const int K = S.K;
    double* eq = A.ev_q;
    double* er = A.ev_r;
    double* eu = A.ev_u;
    double* es = A.ev_s;
    double* et = A.ev_t;
    double* ev = A.ev_v;
    double* ex = A.ev_x;
    for (int k = T::lane(); k < K; k += T::width()) {
      A.th_e[k] = A.sh_th_e[k];
      A.ga_e[k] = A.sh_ga_e[k];
      for (int c = 0; c < 2; ++c) {
        eq[2 * k + c] = A.sh_ev_q[2 * k + c];
        er[2 * k + c] = A.sh_ev_r[2 * k + c];
        eu[2 * k + c] = A.sh_ev_u[2 * k + c];
        es[2 * k + c] = A.sh_ev_s[2 * k + c];
        et[2 * k + c] = A.sh_ev_t[2 * k + c];
        ev[2 * k + c] = A.sh_ev_v[2 * k + c];
        ex[2 * k + c] = A.sh_ev_x[2 * k + c];
      }
    }
    T::sync();
    if (T::lane() == 0) {
      *A.logdet = *A.sh_logdet;
      *A.yCy = *A.sh_yCy;
      *A.ww = *A.sh_ww;
    }
    T::sync();
    S.nevals += 1;
    S.cur_valid = 0;
    return true;
  }

  // Drops component k, shifting those above it down by one.  In chunks of
  // the team's width: the lanes load their entries of a chunk, then store
  // them one place lower (the stores of a chunk lie below the loads of the
  // next).
  SFLS_HD void remove_component(int k) {
    for (int j0 = k; j0 + 1 < S.K; j0 += T::width()) {
      const int j = j0 + T::lane();
      const bool mv = j + 1 < S.K;
      const double t = mv ? A.th[j + 1] : 0.0, g = mv ? A.ga[j + 1] : 0.0;
      T::sync();
      if (mv) {
        A.th[j] = t;
        A.ga[j] = g;
      }
      T::sync();
    }
    T::sync();
    S.K -= 1;
  }

  SFLS_HD int pick_deactivation() const {
    const double thr = (S.zeta > 0.0) ? log((1.0 - S.zeta) / S.zeta) : INFINITY;
    int best = -1;
    double bm = 0.0;
    for (int k = T::lane(); k < S.K; k += T::width()) {
      const double gk = A.ga[k];
      double margin;
      if (!(gk > 0.0)) {
        margin = INFINITY;
      } else {
        const double s = A.ev_s[2 * k];
        const double den = 1.0 - gk * s;
        // sum_g |q~_g|^2 (Woodbury), eq. deactivate / eq. singlecomp-mmv
        double q2t = 0.0;
        for (int gv = 0; gv < A.G; ++gv) {
          const double qr = A.ev_q[gv * A.vk + 2 * k], qi = A.ev_q[gv * A.vk + 2 * k + 1];
          const double t = (qr * qr + qi * qi) / (den * den);
          q2t = gv == 0 ? t : q2t + t;
        }
        const double st = s / den;
        const double lg = A.G == 1 ? log1p(gk * st) : (double)A.G * log1p(gk * st);
        const double lhs = q2t / (1.0 / gk + st) - lg;
        margin = thr - lhs;
      }
      if (margin > 0.0 && (best < 0 || margin > bm)) { best = k; bm = margin; }
    }
    // the largest margin, and the first k with it
    const double gm = T::max(best >= 0 ? bm : -INFINITY);
    best = T::imin((best >= 0 && bm == gm) ? best : INT32_MAX);
    return best == INT32_MAX ? -1 : best;
  }

  // FP64 decision quantities at candidate c (index into cand arrays)
  // (q2 = sum_g |q_g|^2 over the observation vectors)
  SFLS_HD void cand_q2s(int c, double& q2, double& s) const {
    for (int gv = 0; gv < A.G; ++gv) {
      const double qr = A.cand_q[gv * A.vc + 2 * c], qi = A.cand_q[gv * A.vc + 2 * c + 1];
      const double t = qr * qr + qi * qi;
      q2 = gv == 0 ? t : q2 + t;
    }
    s = A.cand_s[c];
  }

  // exact activation decision on cand[0]; returns 1 if a component was added
  SFLS_HD int exact_decide() {
    double q2, s;
    cand_q2s(0, q2, s);
    const double gh = gamma_hat(q2, s, A.G);
    const double gb = (S.K == 0) ? gh : gbar();
    const double dl = delta_L(q2, s, gb, S.zeta, A.G);
    const bool ok = gh > 0.0 && S.zeta > 0.0 && act_criterion(q2, s, gb, S.zeta, P.tau, A.G) &&
                    dl < -P.eps_L;
    if (!ok) return 0;
    if (S.K >= A.kcap || S.K >= Mo) { S.cap_hit = 1; return 0; }
    A.th[S.K] = (double)A.cand[0] / (double)A.L;
    A.ga[S.K] = gh;
    S.K += 1;
    return 1;
  }

  // approximate sweep over cand[1..ncand-1]; returns number added.  The
  // qualifying candidates are taken in increasing (Delta L, grid index)
  // order; each is added unless it lies within approx_min_dist / N of a
  // component.  cbuf_dl / cbuf_gh hold Delta L and gamma_hat per candidate,
  // gamma_hat < 0 marking one that does not qualify or was taken.
  SFLS_HD int approx_decide() {
    const int nc = *A.ncand;
    double q2, s;
    cand_q2s(0, q2, s);
    const double gb0 = (S.K == 0) ? gamma_hat(q2, s, A.G) : gbar();
    const double dlmin = delta_L(q2, s, gb0, S.zeta, A.G);
    const double tau = P.approx_use_tau ? P.tau : 0.0;
    const double gbf = gbar();
    double nq = 0.0;
    for (int c = 1 + T::lane(); c < nc; c += T::width()) {
      double q2c, sc;
      cand_q2s(c, q2c, sc);
      const double gh = gamma_hat(q2c, sc, A.G);
      const double gb = (S.K == 0) ? gh : gbf;
      const double dl = delta_L(q2c, sc, gb, S.zeta, A.G);
      const bool ok = gh > 0.0 && S.zeta > 0.0 && act_criterion(q2c, sc, gb, S.zeta, tau, A.G) &&
                      dl <= dlmin / P.approx_ratio;
      A.cbuf_dl[c] = dl;
      A.cbuf_gh[c] = ok ? gh : -1.0;
      nq += ok ? 1.0 : 0.0;
    }
    T::sync();
    const int m = (int)T::sum(nq);
    int added = 0;
    const double mind = P.approx_min_dist / (double)N;
    for (int i = 0; i < m; ++i) {
      if (S.K >= A.kcap || S.K >= Mo) { S.cap_hit = 1; break; }
      // next qualifying candidate: smallest Delta L, then smallest grid index
      double dlo = INFINITY;
      int lo = INT32_MAX;
      for (int c = 1 + T::lane(); c < nc; c += T::width()) {
        if (!(A.cbuf_gh[c] > 0.0)) continue;
        const double dl = A.cbuf_dl[c];
        const int l = A.cand[c];
        if (dl < dlo || (dl == dlo && l < lo)) { dlo = dl; lo = l; }
      }
      const double dmin = T::min(dlo);
      const int l = T::imin(dlo == dmin ? lo : INT32_MAX);
      int cl = INT32_MAX;  // its candidate slot
      for (int c = 1 + T::lane(); c < nc; c += T::width())
        if (A.cbuf_gh[c] > 0.0 && A.cand[c] == l && A.cbuf_dl[c] == dmin) cl = c;
      cl = T::imin(cl);
      const double gh = A.cbuf_gh[cl];
      T::sync();  // every lane has read the entry before it is marked as taken
      A.cbuf_gh[cl] = -1.0;
      T::sync();
      const double th = (double)l / (double)A.L;
      bool near = false;
      for (int k = T::lane(); k < S.K; k += T::width())
        if (!(wrapd(th, A.th[k]) >= mind)) near = true;
      if (!T::any(near)) {
        A.th[S.K] = th;
        A.ga[S.K] = gh;
        S.K += 1;
        ++added;
      }
    }
    return added;
  }

  // Outputs at the current point: from the evaluation there, or (saved) from
  // q and the objective kept when the last polish step started at it.
  SFLS_HD void finish(bool saved) {
    const int K = S.K;
    const double* q = saved ? A.q_save : A.ev_q;
    T::sync();
    // alpha = gamma .* q at the final point, sorted by theta (stable: the
    // rank of k counts smaller thetas and equal ones before k)
    for (int k = T::lane(); k < K; k += T::width()) {
      const double t = A.th[k];
      int r = 0;
      for (int j = 0; j < K; ++j) {
        const double tj = A.th[j];
        r += (tj < t || (tj == t && j < k)) ? 1 : 0;
      }
      A.out_theta[r] = t;
      A.out_gamma[r] = A.ga[k];
      for (int gv = 0; gv < A.G; ++gv) {  // alpha^(g) = gamma .* q^(g)
        A.out_alpha[gv * A.vo + 2 * r] = A.ga[k] * q[gv * A.vk + 2 * k];
        A.out_alpha[gv * A.vo + 2 * r + 1] = A.ga[k] * q[gv * A.vk + 2 * k + 1];
      }
    }
    *A.out_K = K;
    *A.out_beta = S.beta;
    *A.out_zeta = S.zeta;
    *A.out_obj = (S.yy == 0.0) ? -INFINITY : (saved ? S.f_cur : f_of_eval());
    *A.out_iters = S.it;
    if (A.out_evals) *A.out_evals = S.nevals;
    int st = S.converged ? 0 : 1;
    if (S.cap_hit) st = -5;
    if (S.status != 0) st = S.status;
    *A.out_status = st;
    *A.req = 0;
    S.phase = PH_DONE;
    S.done = 1;
  }

  // -------------------------------------------------------------------------
  // Advance until the next evaluation request (returns) or completion.
  // -------------------------------------------------------------------------
  SFLS_HD void step() {
    enum Lbl {
      L_OUTER, L_EXACT_BEGIN, L_EXACT_DECIDE, L_AFTER_ACT, L_BETA_DO, L_INNER_BEGIN, L_INNER_DIR,
      L_LS_RESULT, L_DEACT_CHECK, L_INNER_END, L_TERM_BEGIN, L_TERM_DO, L_POLISH_BEGIN,
      L_POLISH_STEP, L_FINAL
    };
    int lbl;
    *A.req = 0;
    // a shadow evaluation of this round (granted for the trial requested last)
    bool sh_ready = A.sh_req && (*A.sh_req & 1);
    if (S.phase != PH_START && S.phase != PH_DONE && *A.lev_status != 0) {
      // the factorisation failed at the requested point: stop with what we have
      S.status = -4;
      *A.out_K = S.K;
      for (int k = T::lane(); k < S.K; k += T::width()) {
        A.out_theta[k] = A.th[k];
        A.out_gamma[k] = A.ga[k];
        for (int gv = 0; gv < A.G; ++gv) {
          A.out_alpha[gv * A.vo + 2 * k] = 0.0;
          A.out_alpha[gv * A.vo + 2 * k + 1] = 0.0;
        }
      }
      *A.out_beta = S.beta;
      *A.out_zeta = S.zeta;
      *A.out_obj = NAN;
      *A.out_iters = S.it;
      if (A.out_evals) *A.out_evals = S.nevals;
      *A.out_status = -4;
      S.phase = PH_DONE;
      S.done = 1;
      return;
    }
    switch (S.phase) {
      case PH_DONE:
        return;
      case PH_START: {
        // initialisation (Sec. II-E)
        S.it = 0; S.inner = 0; S.pit = 0; S.K = 0; S.z_changed = 1; S.cur_valid = 0;
        S.converged = 0; S.cap_hit = 0; S.polish = 0; S.mem_n = 0; S.mem_head = 0;
        S.status = 0; S.nevals = 0; S.done = 0; S.saved = 0;
        if (S.yy == 0.0) {
          S.beta = 0.0; S.zeta = 0.0; S.converged = 1;
          lbl = L_FINAL;
          break;
        }
        S.beta = 0.01 * S.yy / (double)Mo;
        S.zeta = 0.2;
        S.eps_beta = P.eps_beta_rel * S.yy / (double)Mo;
        S.approx_on = P.approx_max_iters > 0;
        S.L_prev = INFINITY;
        lbl = L_OUTER;
        break;
      }
      case PH_APPROX_WAIT: {
        S.cur_valid = 1;
        const int added = approx_decide();
        if (added > 0) {
          S.cur_valid = 0;
          S.z_changed = 1;
          lbl = L_AFTER_ACT;
        } else {
          S.approx_on = 0;
          lbl = L_EXACT_DECIDE;  // this grid evaluation is at the current state
        }
        break;
      }
      case PH_EXACT_WAIT: S.cur_valid = 1; lbl = L_EXACT_DECIDE; break;
      case PH_BETA_WAIT: S.cur_valid = 1; lbl = L_BETA_DO; break;
      case PH_INNER_WAIT: S.cur_valid = 1; lbl = L_INNER_DIR; break;
      case PH_LS_WAIT: lbl = L_LS_RESULT; break;
      case PH_DEACT_WAIT: S.cur_valid = 1; lbl = L_DEACT_CHECK; break;
      case PH_TERM_WAIT: S.cur_valid = 1; lbl = L_TERM_DO; break;
      case PH_POLISH_WAIT: S.cur_valid = 1; lbl = L_POLISH_STEP; break;
      default: return;
    }

    for (;;) {
      switch (lbl) {
        case L_OUTER: {
          S.it += 1;
          if (S.it > P.max_outer) { S.it = P.max_outer; lbl = L_POLISH_BEGIN; break; }
          if (S.approx_on && S.it <= P.approx_max_iters && S.zeta > 0.0) {
            request_current(2 | 4 | 1);  // GRID | APPROX | EVAL
            S.phase = PH_APPROX_WAIT;
            return;
          }
          S.approx_on = S.approx_on && S.it <= P.approx_max_iters && S.zeta > 0.0;
          lbl = L_EXACT_BEGIN;
          break;
        }
        case L_EXACT_BEGIN: {
          if (!(S.zeta > 0.0)) { lbl = L_AFTER_ACT; break; }  // nothing can activate
          request_current(2 | 1);
          S.phase = PH_EXACT_WAIT;
          return;
        }
        case L_EXACT_DECIDE: {
          if (exact_decide()) {
            S.cur_valid = 0;
            S.z_changed = 1;
            lbl = L_EXACT_BEGIN;
          } else {
            lbl = L_AFTER_ACT;
          }
          break;
        }
        case L_AFTER_ACT: {
          const double zn = (double)S.K / (double)Mo;  // eq. zetaUpdate
          S.zeta = zn < 0.5 ? zn : 0.5;
          if (!S.cur_valid) {
            request_current(1);
            S.phase = PH_BETA_WAIT;
            return;
          }
          lbl = L_BETA_DO;
          break;
        }
        case L_BETA_DO: {
          // eq. betaUpdate with mu = gamma.q, tr = beta sum gamma s, ||y - A mu||^2 = beta^2 ||w||^2
          double tr = 0.0;
          for (int k = T::lane(); k < S.K; k += T::width()) tr += A.ga[k] * A.ev_s[2 * k];
          tr = T::sum(tr);
          // with G vectors (Sec. V): (G beta tr + beta^2 sum_g ||w_g||^2) / (G M)
          double bn = A.G == 1
                          ? (S.beta * tr + S.beta * S.beta * (*A.ww)) / (double)Mo
                          : ((double)A.G * S.beta * tr + S.beta * S.beta * (*A.ww)) /
                                ((double)A.G * (double)Mo);
          if (!(bn > S.eps_beta)) bn = S.eps_beta;
          if (bn != S.beta) { S.beta = bn; S.cur_valid = 0; }
          if (S.z_changed) { mem_reset(); S.z_changed = 0; }
          S.inner = 0;
          lbl = L_INNER_BEGIN;
          break;
        }
        case L_INNER_BEGIN: {
          if (S.inner >= P.max_inner || S.K == 0) { lbl = L_TERM_BEGIN; break; }
          if (!S.cur_valid) {
            request_current(1);
            S.phase = PH_INNER_WAIT;
            return;
          }
          lbl = L_INNER_DIR;
          break;
        }
        case L_INNER_DIR: {
          const int n = 2 * S.K;
          derivs(A.ga, A.g, A.gt);  // gt used as h scratch
          direction(A.g, A.gt, A.d, n);
          S.lam2 = -dot(A.g, A.d, n);
          S.f_cur = f_of_eval();
          ls_begin(false);
          ls_request();
          S.phase = PH_LS_WAIT;
          return;
        }
        case L_LS_RESULT: {
          const double ft = f_of_eval();
          bool accept = ft <= S.f_cur + P.ls_c1 * S.alpha * S.gd;
          // polish: within the objective's rounding level, a step is judged by
          // the diagonal Newton decrement instead
          if (!accept && S.polish && ft <= S.f_cur + P.polish_ftol * (1.0 + fabs(S.f_cur)))
            accept = newton_dec(A.ga_e) < S.nu0;
          if (accept) {
            // accept: pair (alpha d, g_t - g), move to the trial point
            const int K = S.K, n = 2 * K;
            derivs(A.ga_e, A.gt, nullptr);
            for (int e = T::lane(); e < n; e += T::width()) {
              A.gt[e] -= A.g[e];
              A.d[e] *= S.alpha;
            }
            mem_push(A.d, A.gt, n);
            double maxdth = 0.0;
            for (int k = T::lane(); k < K; k += T::width()) {
              maxdth = fmax(maxdth, fabs(A.d[k]));
              A.th[k] = A.th_e[k];
              A.ga[k] = A.ga_e[k];
            }
            T::sync();
            maxdth = T::max(maxdth);
            S.cur_valid = 1;
            if (S.polish) {
              S.pit += 1;
              if (maxdth < P.polish_tol / (double)N) { lbl = L_FINAL; break; }
              lbl = L_POLISH_STEP;
              break;
            }
            lbl = L_DEACT_CHECK;
            break;
          }
          S.alpha *= 0.5;
          S.ls_trial += 1;
          bool give_up = S.ls_trial >= P.ls_max;
          if (S.polish && !give_up) {
            // the polish stops once the shortened step moves no frequency by
            // the polish tolerance
            double dmax = 0.0;
            for (int k = T::lane(); k < S.K; k += T::width()) dmax = fmax(dmax, fabs(A.d[k]));
            dmax = T::max(dmax);
            give_up = S.alpha * dmax < P.polish_tol / (double)N;
          }
          if (!S.polish && !give_up) {
            // the inner search stops once the decrease it requires is below the
            // rounding level of the objective
            give_up = P.ls_c1 * S.alpha * fabs(S.gd) < P.polish_ftol * (1.0 + fabs(S.f_cur));
          }
          if (give_up) {
            // line search failed: current point unchanged (needs re-evaluation)
            if (S.polish) { lbl = L_FINAL; break; }
            lbl = L_TERM_BEGIN;
            break;
          }
          if (sh_ready) {
            sh_ready = false;
            if (take_shadow()) { lbl = L_LS_RESULT; break; }
          }
          ls_request();
          S.phase = PH_LS_WAIT;
          return;
        }
        case L_DEACT_CHECK: {
          const int k = pick_deactivation();
          if (k >= 0) {
            remove_component(k);
            mem_reset();
            S.cur_valid = 0;
            request_current(1);
            S.phase = PH_DEACT_WAIT;
            return;
          }
          lbl = L_INNER_END;
          break;
        }
        case L_INNER_END: {
          S.inner += 1;
          if (S.lam2 < gN() * P.tol_newton) { lbl = L_TERM_BEGIN; break; }
          lbl = L_INNER_BEGIN;
          break;
        }
        case L_TERM_BEGIN: {
          if (!S.cur_valid) {
            request_current(1);
            S.phase = PH_TERM_WAIT;
            return;
          }
          lbl = L_TERM_DO;
          break;
        }
        case L_TERM_DO: {
          const double Lc = f_of_eval();
          if (fabs(Lc - S.L_prev) < gN() * P.tol_obj) {
            S.converged = 1;
            lbl = L_POLISH_BEGIN;
            break;
          }
          S.L_prev = Lc;
          lbl = L_OUTER;
          break;
        }
        case L_POLISH_BEGIN: {
          mem_reset();
          S.pit = 0;
          if (!S.cur_valid) {
            request_current(1);
            S.phase = PH_POLISH_WAIT;
            return;
          }
          lbl = L_POLISH_STEP;
          break;
        }
        case L_POLISH_STEP: {
          if (S.pit >= P.polish_max_iters || S.K == 0) { lbl = L_FINAL; break; }
          const int n = 2 * S.K;
          derivs(A.ga, A.g, A.gt);
          double nu = 0.0;
          for (int e = T::lane(); e < n; e += T::width()) nu += A.g[e] * A.g[e] / A.gt[e];
          S.nu0 = T::sum(nu);
          direction(A.g, A.gt, A.d, n);
          S.f_cur = f_of_eval();
          for (int gv = 0; gv < A.G; ++gv)
            for (int e = T::lane(); e < n; e += T::width())
              A.q_save[gv * A.vk + e] = A.ev_q[gv * A.vk + e];
          S.saved = 1;
          ls_begin(true);
          ls_request();
          S.phase = PH_LS_WAIT;
          return;
        }
        case L_FINAL: {
          if (!S.cur_valid && S.yy != 0.0) {
            if (S.polish && S.saved) {
              // the polish's last line search failed: the current point is the
              // one its step started from
              finish(true);
              return;
            }
            request_current(1);
            S.phase = PH_POLISH_WAIT;
            S.pit = P.polish_max_iters;  // resumes into L_POLISH_STEP -> L_FINAL
            return;
          }
          finish(false);
          return;
        }
        default:
          return;
      }
    }
  }
};

}  // namespace sfls
