// a6: q^G and s^G on the grid theta_l = l/L, and Delta L;  a7: selection
// (argmin for the exact activation step, local minima for the approximate
// scheme).
#include "sfls_kernels.hpp"
#include "k_launch.hpp"

namespace sfls {

constexpr int GRID_NT = 256;
constexpr int GRID_ANCHOR = 4;  // points per thread between exact residue twiddles
constexpr int SEL_NT = 1024;
constexpr int SEL_COLLECT = 2048;  // local minima gathered before sorting

template <typename R> __device__ __forceinline__ R rinf();
template <> __device__ __forceinline__ double rinf<double>() { return __builtin_inf(); }
template <> __device__ __forceinline__ float rinf<float>() { return __builtin_inff(); }

// Delta L of eq. delta_L at one grid point in precision R.  gb > 0: fixed
// average variance; gb <= 0: the per-point optimum of eq. activate_gamma
// (empty active set), for which Delta L = ln(kappa odds) - (kappa - 1).
// With G observation vectors (Sec. V, eq. singlecomp-mmv) q2 is sum_g |q_g|^2
// and Delta L = G ln(1 + gb s) + ln odds - q2 / (1/gb + s), or with the
// per-point optimum G (ln kap - (kap - 1)) + ln odds, kap = q2 / (G s); both are
// written so that G = 1 performs the single-vector operations.
template <typename R>
__device__ __forceinline__ R delta_L_point(R q2, R s, R gb, R odds, int G = 1) {
  if (!(s > (R)0)) return rinf<R>();
  if (gb > (R)0) {
    const R lg = log(fma(gb, s, (R)1) * odds);
    return (G == 1 ? lg : lg + (R)(G - 1) * log1p(gb * s)) - q2 / ((R)1 / gb + s);
  }
  const R kap = (G == 1 ? q2 : q2 / (R)G) / s;
  if (kap > (R)1)
    return G == 1 ? log(kap * odds) - (kap - (R)1)
                  : log(kap * odds) + (R)(G - 1) * log(kap) - (R)G * (kap - (R)1);
  return log(odds);
}

// ---------------------------------------------------------------------------
// a6.  Grid of L = R M points split by residue r = l mod R (M a power of
// two, min(2^ceil(log2 N), cap)):  with l = R f + r,
//   q^G_l = sum_m [sum_{n = m mod M} w_n e^{-j2pi n r/L}] e^{-j2pi m f/M}   (M-point DFT)
//   s^G_l = sum_m [sum_{i = m mod M} omega_s(i) e^{j2pi i r/L}] e^{+j2pi m f/M}
// (n over 0..N-1, i over -N+1..N-1; the inner sums fold the inputs onto M points)
// so each workgroup (instance, r) runs two M-point FFTs in LDS (padded layout).  The
// residue twiddles come from exact fractions (n r mod L)/L.  Outputs per
// point: optional q^G, s^G, Delta L; always a per-workgroup argmin
// (lowest l on ties).  Blocks of one instance sit on one XCD:
// blockIdx.x = xcd + 8 j  ->  instance-group j/R... see host mapping.
//
// DER = true: the theta-derivative arrays of the same transforms (Sec. III-D,
// eqs. r and t on the grid),
//   r^G_l = sum_n 2 pi n w_n e^{-j2pi n l/L},   t^G_l = sum_i omega_t(i) e^{+j2pi i l/L},
// with w scaled by D = diag(2 pi n) on the way in and omega_t (the diagonal
// sums of D C^{-1}, lag i at omt[ooff + i + N - 1]) in place of omega_s; t^G
// is complex.  No Delta L and no argmin.
// ---------------------------------------------------------------------------
template <typename R, bool DER>
__global__ __launch_bounds__(GRID_NT) void k_grid(const InstInfo* __restrict__ info,
                                                  const int32_t* __restrict__ req,
                                                  const cd* __restrict__ w,
                                                  const cd* __restrict__ oms,
                                                  const double* __restrict__ gbar,
                                                  const double* __restrict__ zeta,
                                                  const typename cpx<R>::T* __restrict__ tw,
                                                  int logtw, int Rmax, int B,
                                                  typename cpx<R>::T* __restrict__ qG,
                                                  R* __restrict__ sG, R* __restrict__ dL,
                                                  double* __restrict__ part_val,
                                                  int64_t* __restrict__ part_idx,
                                                  typename cpx<R>::T* __restrict__ tG,
                                                  Vecs vv) {
  using C = typename cpx<R>::T;
  // XCD-aware mapping: consecutive block ids go round-robin over 8 XCDs; give
  // all residues of one instance the same id mod 8 so they share an L2.
  const int id = blockIdx.x;
  const int xcd = id & 7, slot = id >> 3;
  const int bi = xcd + 8 * (slot / Rmax);
  const int r = slot % Rmax;
  if (bi >= B) return;
  if (req && !(req[bi] & REQ_GRID)) return;
  const InstInfo in = info[bi];
  if (r >= in.R) {
    if (!DER && threadIdx.x == 0) { part_val[(int64_t)bi * Rmax + r] = __builtin_inf(); part_idx[(int64_t)bi * Rmax + r] = -1; }
    return;
  }
  const int N = in.N, M = in.M, logM = in.logM, L = in.L, P = in.P;
  extern __shared__ unsigned char smem[];
  C* lq = reinterpret_cast<C*>(smem);  // padded layout
  C* ls = lq + padded(M);
  __shared__ C s_tw[FFT_TWL];
  __shared__ double rv[GRID_NT / 64];
  __shared__ int64_t ri[GRID_NT / 64];
  const int tid = threadIdx.x;
  load_tw_head<GRID_NT>(s_tw, tw);
  const cd* wb = w + in.off;
  // lag i of the second input: omega_s in the convolution layout (i mod P),
  // or omega_t in the natural layout (i + N - 1)
  const cd* ob = !oms ? nullptr : (DER ? oms + in.ooff + (N - 1) : oms + in.poff);
  // (DER without omega_t: r^G alone, the second transform runs on zeros)
  const bool has2 = !DER || oms != nullptr;
  auto lag = [&](int i) -> cd {
    return !has2 ? cd{0.0, 0.0} : (DER ? ob[i] : ob[(i + P) & (P - 1)]);
  };
  // the first input: w, or D w
  auto wn = [&](int n) -> cd { return DER ? cscale(wb[n], 6.283185307179586 * (double)n) : wb[n]; };
  // M >= N: the residue twiddles exp(j 2 pi m r / L) of a thread's points m =
  // tid + GRID_NT j come from an exact fraction every GRID_ANCHOR-th point and
  // rotations by exp(j 2 pi GRID_NT r / L) in between; the lag m - M takes the
  // same twiddle times exp(-j 2 pi M r / L)
  const cd rotg = cis_frac(((int64_t)GRID_NT * r) % L, L);
  const cd cM = cconj(cis_frac(((int64_t)M * r) % L, L));
  // vectors g >= 1 of a multiple-vector launch: q^G only, into lq
  auto load_q = [&](const cd* __restrict__ wv) {
    cd e1{1.0, 0.0};
    int jq = 0;
    for (int m = tid; m < M; m += GRID_NT, ++jq) {
      cd qv{0.0, 0.0};
      if (M >= N) {
        e1 = (jq % GRID_ANCHOR == 0) ? cis_frac(((int64_t)m * r) % L, L) : cmul(e1, rotg);
        if (m < N) qv = cmul(wv[m], cconj(e1));
      } else {
        for (int n = m; n < N; n += M) qv = cfma(wv[n], cconj(cis_frac(((int64_t)n * r) % L, L)), qv);
      }
      lq[pidx(m)] = C{(decltype(C{}.x))qv.x, (decltype(C{}.x))qv.y};
    }
  };
  cd e{1.0, 0.0};
  int jt = 0;
  for (int m = tid; m < M; m += GRID_NT, ++jt) {
    cd qv{0.0, 0.0}, sv{0.0, 0.0};
    if (M >= N) {
      // one sample and at most two lags (m and m - M) per point
      e = (jt % GRID_ANCHOR == 0) ? cis_frac(((int64_t)m * r) % L, L) : cmul(e, rotg);
      if (m < N) {
        qv = cmul(wn(m), cconj(e));
        sv = cmul(lag(m), e);
      }
      const int i2 = m - M;
      if (i2 > -N) sv = cfma(lag(i2), cmul(e, cM), sv);
    } else {
      for (int n = m; n < N; n += M) qv = cfma(wn(n), cconj(cis_frac(((int64_t)n * r) % L, L)), qv);
      // lags i = m mod M in (-N, N), from the most negative one up
      for (int i = m - M * ((m + N - 1) / M); i < N; i += M) {
        const int64_t ph = (((int64_t)i % L + L) % L) * r % L;
        sv = cfma(lag(i), cis_frac(ph, L), sv);
      }
    }
    lq[pidx(m)] = C{(decltype(C{}.x))qv.x, (decltype(C{}.x))qv.y};
    ls[pidx(m)] = C{(decltype(C{}.x))sv.x, (decltype(C{}.x))sv.y};
  }
  __syncthreads();
  dif_fftn<GRID_NT>(lq, ls, 2, logM, false, true, (const C*)s_tw, tw);
  if (DER) {
    for (int p = tid; p < M; p += GRID_NT) {
      const int64_t l = (int64_t)bitrev(p, logM) * in.R + r;
      if (qG) qG[in.goff + l] = lq[pidx(p)];
      if (tG) tG[in.goff + l] = ls[pidx(p)];
    }
    return;
  }
  const int G = DER ? 1 : vv.G;
  if (G > 1) {
    // sum_g |q^G_g|^2 in the imaginary part of the s^G buffer (s^G is real);
    // q^G of vector 0 stays in lq for the output
    for (int p = tid; p < M; p += GRID_NT) ls[pidx(p)].y = cabs2(lq[pidx(p)]);
    for (int gv = 1; gv < G; ++gv) {
      // lq of vector 0 was read by this thread only; the transforms below
      // exchange data across the block
      if (gv == 1 && qG) {
        for (int p = tid; p < M; p += GRID_NT)
          qG[in.goff + (int64_t)bitrev(p, logM) * in.R + r] = lq[pidx(p)];
      }
      __syncthreads();
      load_q(w + gv * vv.wstride + in.off);
      __syncthreads();
      dif_fftn<GRID_NT>(lq, lq, 1, logM, false, false, (const C*)s_tw, tw);
      for (int p = tid; p < M; p += GRID_NT) ls[pidx(p)].y += cabs2(lq[pidx(p)]);
    }
    __syncthreads();
  }
  // gbar and zeta may be absent when neither Delta L nor its argmin is wanted
  const R gb = gbar ? (R)gbar[bi] : (R)1;
  const double z = zeta ? zeta[bi] : 0.5;
  const R odds = (R)((1.0 - z) / z);
  double best = __builtin_inf();
  int64_t bidx = INT64_MAX;
  for (int p = tid; p < M; p += GRID_NT) {
    const int f = bitrev(p, logM);
    const int64_t l = (int64_t)f * in.R + r;
    const C qv = lq[pidx(p)];
    const R sv = ls[pidx(p)].x;
    const R q2 = G > 1 ? ls[pidx(p)].y : cabs2(qv);
    R d = delta_L_point<R>(q2, sv, gb, odds, G);
    if (d != d) d = rinf<R>();
    if (qG && G == 1) qG[in.goff + l] = qv;
    if (sG) sG[in.goff + l] = sv;
    if (dL) dL[in.goff + l] = d;
    const double dd = (double)d;
    if (dd < best || (dd == best && l < bidx)) { best = dd; bidx = l; }
  }
  // block argmin, lowest index on ties
  const int lane = tid & 63, wv = tid >> 6;
  for (int o = 32; o >= 1; o >>= 1) {
    const double ov = __shfl_xor(best, o);
    const int64_t oi = __shfl_xor(bidx, o);
    if (ov < best || (ov == best && oi < bidx)) { best = ov; bidx = oi; }
  }
  if (lane == 0) { rv[wv] = best; ri[wv] = bidx; }
  __syncthreads();
  if (tid == 0) {
    for (int k = 1; k < GRID_NT / 64; ++k)
      if (rv[k] < best || (rv[k] == best && ri[k] < bidx)) { best = rv[k]; bidx = ri[k]; }
    part_val[(int64_t)bi * Rmax + r] = best;
    part_idx[(int64_t)bi * Rmax + r] = bidx;
  }
}

// ---------------------------------------------------------------------------
// a7.  Selection, one workgroup per instance.
//   exact:        cand[0] = argmin over the residue partials (lowest l).
//   approximate:  cand[0] = argmin; cand[1..] = local minima of Delta L
//                 (cyclic neighbours, <= on both sides) with
//                 Delta L <= Delta L_min / ratio + slack, sorted by
//                 (Delta L, l), at most cand_cap of them.
// The slack keeps every point the FP64 re-check could accept when the grid is
// FP32.  ncand[b] = number of entries written; overflow[b] = 1 if more local
// minima passed the pre-filter than could be kept.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(SEL_NT) void k_select(const InstInfo* __restrict__ info,
                                                   const int32_t* __restrict__ req,
                                                   const R* __restrict__ dL, int Rmax,
                                                   const double* __restrict__ part_val,
                                                   const int64_t* __restrict__ part_idx,
                                                   double approx_ratio, double slack_rel,
                                                   int cand_cap, int32_t* __restrict__ cand,
                                                   int32_t* __restrict__ ncand,
                                                   int32_t* __restrict__ overflow) {
  const int bi = blockIdx.x;
  if (!(req[bi] & REQ_GRID)) return;
  const InstInfo in = info[bi];
  const int tid = threadIdx.x;
  __shared__ double best_v;
  __shared__ int64_t best_i;
  __shared__ double key_d[SEL_COLLECT];
  __shared__ int32_t key_l[SEL_COLLECT];
  __shared__ int cnt;
  if (tid == 0) {
    double bv = __builtin_inf();
    int64_t bx = INT64_MAX;
    for (int r = 0; r < in.R; ++r) {
      const double v = part_val[(int64_t)bi * Rmax + r];
      const int64_t ix = part_idx[(int64_t)bi * Rmax + r];
      if (v < bv || (v == bv && ix < bx)) { bv = v; bx = ix; }
    }
    if (bx == INT64_MAX) bx = 0;
    best_v = bv;
    best_i = bx;
    cnt = 0;
  }
  __syncthreads();
  int32_t* cb = cand + in.coff;
  if (!(req[bi] & REQ_APPROX)) {
    if (tid == 0) { cb[0] = (int32_t)best_i; ncand[bi] = 1; overflow[bi] = 0; }
    return;
  }
  const double dmin = best_v;
  const int L = in.L;
  const R* d = dL + in.goff;
  if (dmin < 0.0) {
    const double thr = dmin / approx_ratio + slack_rel * fabs(dmin);
    for (int l = tid; l < L; l += SEL_NT) {
      const double v = (double)d[l];
      if (!(v <= thr)) continue;
      const double vl = (double)d[(l - 1 + L) & (L - 1)];
      const double vr = (double)d[(l + 1) & (L - 1)];
      if (v <= vl && v <= vr) {
        const int slot = atomicAdd(&cnt, 1);
        if (slot < SEL_COLLECT) { key_d[slot] = v; key_l[slot] = l; }
      }
    }
  }
  __syncthreads();
  const int total = cnt;
  const int kept = min(total, SEL_COLLECT);
  // bitonic sort of (value, index) over the next power of two
  int n2 = 1;
  while (n2 < kept) n2 <<= 1;
  for (int i = kept + tid; i < n2; i += SEL_NT) { key_d[i] = __builtin_inf(); key_l[i] = INT32_MAX; }
  __syncthreads();
  for (int k = 2; k <= n2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < n2; i += SEL_NT) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const bool up = (i & k) == 0;
          const double a = key_d[i], b2 = key_d[ixj];
          const int la = key_l[i], lb = key_l[ixj];
          const bool gt = (a > b2) || (a == b2 && la > lb);
          if (gt == up) { key_d[i] = b2; key_d[ixj] = a; key_l[i] = lb; key_l[ixj] = la; }
        }
      }
      __syncthreads();
    }
  }
  const int nout = min(kept, cand_cap);
  if (tid == 0) { cb[0] = (int32_t)best_i; ncand[bi] = 1 + nout; overflow[bi] = (total > nout) ? 1 : 0; }
  for (int i = tid; i < nout; i += SEL_NT) cb[1 + i] = key_l[i];
}

// argmin over the residue partials (lowest l on ties) for the API call
__global__ void k_argmin_out(const InstInfo* __restrict__ info, int Rmax,
                             const double* __restrict__ part_val,
                             const int64_t* __restrict__ part_idx, int64_t* __restrict__ amin,
                             double* __restrict__ aval, int B) {
  const int bi = blockIdx.x * blockDim.x + threadIdx.x;
  if (bi >= B) return;
  const int R = info[bi].R;
  double bv = __builtin_inf();
  int64_t bx = INT64_MAX;
  for (int r = 0; r < R; ++r) {
    const double v = part_val[(int64_t)bi * Rmax + r];
    const int64_t ix = part_idx[(int64_t)bi * Rmax + r];
    if (v < bv || (v == bv && ix < bx)) { bv = v; bx = ix; }
  }
  if (bx == INT64_MAX) bx = 0;
  if (amin) amin[bi] = bx;
  if (aval) aval[bi] = bv;
}

hipError_t launch_argmin_out(const InstInfo* info, int Rmax, const double* part_val,
                             const int64_t* part_idx, int64_t* amin, double* aval, int B,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_argmin_out, dim3((B + 63) / 64), dim3(64), 0, st, info, Rmax, part_val,
                     part_idx, amin, aval, B);
  return hipGetLastError();
}

template <typename R, bool DER>
static void launch_grid_t(dim3 grid, int maxM, hipStream_t st, const InstInfo* info,
                          const int32_t* req, const cd* w, const cd* oms, const double* gbar,
                          const double* zeta, const void* tw, int logtw, int Rmax, int B, void* qG,
                          void* sG, void* dL, double* part_val, int64_t* part_idx, void* tG,
                          Vecs vv = Vecs{}) {
  using C = typename cpx<R>::T;
  const size_t shm = 2 * (size_t)padded(maxM) * sizeof(C);
  (void)hipFuncSetAttribute((const void*)k_grid<R, DER>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)shm);
  hipLaunchKernelGGL((k_grid<R, DER>), grid, dim3(GRID_NT), shm, st, info, req, w, oms, gbar, zeta,
                     (const C*)tw, logtw, Rmax, B, (C*)qG, (R*)sG, (R*)dL, part_val, part_idx,
                     (C*)tG, vv);
}

hipError_t launch_grid(int prec, const InstInfo* info, const int32_t* req, const cd* w,
                       const cd* oms, const double* gbar, const double* zeta, const void* tw,
                       int logtw, int Rmax, int B, int maxM, void* qG, void* sG, void* dL,
                       double* part_val, int64_t* part_idx, hipStream_t st, Vecs vv) {
  const int nslots = ((B + 7) / 8) * Rmax;  // per XCD
  dim3 grid(8 * nslots);
  if (prec == 0)
    launch_grid_t<double, false>(grid, maxM, st, info, req, w, oms, gbar, zeta, tw, logtw, Rmax, B,
                                 qG, sG, dL, part_val, part_idx, nullptr, vv);
  else
    launch_grid_t<float, false>(grid, maxM, st, info, req, w, oms, gbar, zeta, tw, logtw, Rmax, B,
                                qG, sG, dL, part_val, part_idx, nullptr, vv);
  return hipGetLastError();
}

hipError_t launch_grid_deriv(int prec, const InstInfo* info, const int32_t* req, const cd* w,
                             const cd* omt, const void* tw, int logtw, int Rmax, int B, int maxM,
                             void* rG, void* tG, hipStream_t st) {
  const int nslots = ((B + 7) / 8) * Rmax;
  dim3 grid(8 * nslots);
  if (prec == 0)
    launch_grid_t<double, true>(grid, maxM, st, info, req, w, omt, nullptr, nullptr, tw, logtw,
                                Rmax, B, rG, nullptr, nullptr, nullptr, nullptr, tG);
  else
    launch_grid_t<float, true>(grid, maxM, st, info, req, w, omt, nullptr, nullptr, tw, logtw,
                               Rmax, B, rG, nullptr, nullptr, nullptr, nullptr, tG);
  return hipGetLastError();
}

hipError_t launch_select(int prec, const InstInfo* info, const int32_t* req, const void* dL,
                         int Rmax, const double* part_val, const int64_t* part_idx,
                         double approx_ratio, double slack_rel, int cand_cap, int32_t* cand,
                         int32_t* ncand, int32_t* overflow, int B, hipStream_t st) {
  if (prec == 0)
    hipLaunchKernelGGL(k_select<double>, dim3(B), dim3(SEL_NT), 0, st, info, req,
                       (const double*)dL, Rmax, part_val, part_idx, approx_ratio, slack_rel,
                       cand_cap, cand, ncand, overflow);
  else
    hipLaunchKernelGGL(k_select<float>, dim3(B), dim3(SEL_NT), 0, st, info, req,
                       (const float*)dL, Rmax, part_val, part_idx, approx_ratio, slack_rel,
                       cand_cap, cand, ncand, overflow);
  return hipGetLastError();
}

}  // namespace sfls
