// a8: q, r, u, s, t, v, x at the active frequencies (and q, s at grid
// candidates for the FP64 re-check of activation decisions).
#include "sfls_kernels.hpp"
#include "k_launch.hpp"

namespace sfls {

constexpr int ACT_NT = 256;
constexpr int ACT_ANCHOR = 4;  // samples per thread between exact phase evaluations
constexpr int NU_NT = 512;

// Whether instance work of npts points at N samples uses the NUFFT form below
// (mode: 0 automatic, 1 never, 2 always); 4 npts <= 3 P keeps its per-point
// storage inside the instance's scratch blocks 1-3.
__device__ __forceinline__ bool use_nufft(int mode, int N, int P, int npts) {
  if (mode == 1 || npts <= 0 || 4 * npts > 3 * P) return false;
  if (mode == 2) return true;
  return N >= 512 && (double)npts * (double)N >= NU_MIN_WORK;
}

// Instances of at most ACT_LDS_N samples whose points take the direct sums
// run in k_active_lds (w and rho staged once in LDS, one wave per point)
// instead of the item-parallel k_active.
constexpr int ACT_LDS_N = 4096;
__device__ __forceinline__ bool use_lds_active(int mode, int N, int P, int npts) {
  return npts > 0 && N <= ACT_LDS_N && !use_nufft(mode, N, P, npts);
}

// Exclusive prefix over instances of the number of work items:
// items(b) = (EVAL ? K[b] : 0) + (GRID ? ncand[b] : 0).  prefix has B+1 entries.
__global__ __launch_bounds__(1024) void k_item_scan(const InstInfo* __restrict__ info,
                                                    const int32_t* __restrict__ req,
                                                    const int32_t* __restrict__ Keval,
                                                    const int32_t* __restrict__ ncand, int B,
                                                    int nmode, int32_t* __restrict__ prefix) {
  __shared__ int32_t part[1024];
  const int tid = threadIdx.x;
  const int per = (B + 1023) / 1024;
  const int b0 = tid * per;
  // instances handled by the NUFFT kernel contribute no items here
  auto items = [&](int b) {
    const int32_t rq = req[b];
    const int n = ((rq & REQ_EVAL) ? Keval[b] : 0) + ((rq & REQ_GRID) && ncand ? ncand[b] : 0);
    return (use_nufft(nmode, info[b].N, info[b].P, n) || use_lds_active(nmode, info[b].N, info[b].P, n))
               ? 0 : n;
  };
  int32_t loc = 0;
  for (int b = b0; b < min(B, b0 + per); ++b) loc += items(b);
  part[tid] = loc;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int32_t v = (tid >= o) ? part[tid - o] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int32_t run = part[tid] - loc;  // exclusive
  for (int b = b0; b < min(B, b0 + per); ++b) {
    prefix[b] = run;
    run += items(b);
  }
  if (tid == 1023) prefix[B] = part[1023];
}

// Outputs of point j from its 14 sums (q, n q, n^2 q, then G_0..G_3 as
// re/im pairs): q, r, u and s, t, v, x by the separable form (full points),
// or q and s (grid candidates, j >= nk).
__device__ __forceinline__ void active_out(const double (&acc)[14], bool full, const InstInfo& in,
                                           int j, int nk, double idl, const SepCoef& cf, cd* oq,
                                           cd* orr, cd* ou, cd* os, cd* ot, cd* ov, cd* ox,
                                           cd* cq, double* cs) {
  const double TWO_PI = 6.283185307179586476925286766559;
  const cd G[4] = {cd{acc[6], acc[7]}, cd{acc[8], acc[9]}, cd{acc[10], acc[11]},
                   cd{acc[12], acc[13]}};
  const int nq = full ? 4 : 1;
  cd outv[4];
  for (int qk = 0; qk < nq; ++qk) {
    const double* C = cf.c[qk];
    const int am = (qk == 0) ? 1 : 3;
    cd a2{0.0, 0.0};
    for (int a = 0; a <= am; ++a)
      for (int b2 = 0; b2 <= am; ++b2) {
        const double cab = C[a * 4 + b2];
        if (cab != 0.0) {
          const cd pr = cmulc(G[a], G[b2]);
          a2.x = fma(cab, pr.x, a2.x);
          a2.y = fma(cab, pr.y, a2.y);
        }
      }
    outv[qk] = cscale(a2, idl);
  }
  const cd q{acc[0], acc[1]};
  if (full) {
    const int64_t o = in.koff + j;
    oq[o] = q;
    orr[o] = cd{TWO_PI * acc[2], TWO_PI * acc[3]};
    ou[o] = cd{TWO_PI * TWO_PI * acc[4], TWO_PI * TWO_PI * acc[5]};
    os[o] = cd{outv[0].x, 0.0};
    ot[o] = outv[1];
    ov[o] = outv[2];
    ox[o] = outv[3];
  } else {
    const int64_t o = in.coff + (j - nk);
    cq[o] = q;
    cs[o] = outv[0].x;
  }
}

// q, r, u of observation vector gv >= 1 at point j from its six sums (q, n q,
// n^2 q as re/im pairs); grid candidates (j >= nk) keep q only.
__device__ __forceinline__ void vec_out(const double (&a)[6], bool full, const InstInfo& in, int j,
                                        int nk, int gv, const Vecs& vv, cd* oq, cd* orr, cd* ou,
                                        cd* cq) {
  const double TWO_PI = 6.283185307179586476925286766559;
  if (full) {
    const int64_t o = gv * vv.kstride + in.koff + j;
    oq[o] = cd{a[0], a[1]};
    orr[o] = cd{TWO_PI * a[2], TWO_PI * a[3]};
    ou[o] = cd{TWO_PI * TWO_PI * a[4], TWO_PI * TWO_PI * a[5]};
  } else {
    cq[gv * vv.cstride + in.coff + (j - nk)] = cd{a[0], a[1]};
  }
}

// ---------------------------------------------------------------------------
// With e_n = exp(-j 2 pi n theta) and x_n = n - c, c = (N-1)/2:
//   q = sum w_n e_n,  r = 2 pi sum n w_n e_n,  u = (2 pi)^2 sum n^2 w_n e_n
//   G_a = sum x_n^a rho_n e_n                     (a = 0..3)
//   s, t, v, x = delta^{-1} sum_ab C[a][b] G_a conj(G_b)
// The last line is the diagonal-sum series of eq. sFourier with the
// Appendix-B weights written as polynomials in (q, q + i): the double sum
// over (q, q+i) factorises into the product of two single sums.
// Work items are distributed over a fixed grid (block g takes g, g+G, ...).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(ACT_NT) void k_active(const InstInfo* __restrict__ info,
                                                   const int32_t* __restrict__ req,
                                                   const int32_t* __restrict__ Keval,
                                                   const int32_t* __restrict__ prefix, int B,
                                                   const double* __restrict__ theta,
                                                   const int32_t* __restrict__ cand,
                                                   const cd* __restrict__ w,
                                                   const cd* __restrict__ rho,
                                                   const double* __restrict__ delta,
                                                   const SepCoef* __restrict__ coef,
                                                   cd* __restrict__ oq, cd* __restrict__ orr,
                                                   cd* __restrict__ ou, cd* __restrict__ os,
                                                   cd* __restrict__ ot, cd* __restrict__ ov,
                                                   cd* __restrict__ ox, cd* __restrict__ cq,
                                                   double* __restrict__ cs, Vecs vv) {
  __shared__ double red[14 * (ACT_NT / 64)];
  const int total = prefix[B];
  const int tid = threadIdx.x;
  const double TWO_PI = 6.283185307179586476925286766559;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    int lo = 0, hi = B;  // prefix[lo] <= item < prefix[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (prefix[mid] <= item) lo = mid; else hi = mid;
    }
    const int bi = lo;
    const InstInfo in = info[bi];
    const int nk = (req[bi] & REQ_EVAL) ? Keval[bi] : 0;
    const int j = item - prefix[bi];
    const bool full = j < nk;
    const double th = full ? theta[in.koff + j]
                           : (double)cand[in.coff + (j - nk)] / (double)in.L;
    const int N = in.N;
    const double cN = 0.5 * (double)(N - 1);
    const cd* wb = w + in.off;
    const cd* rb = rho + in.off;
    double acc[14];
#pragma unroll
    for (int i = 0; i < 14; ++i) acc[i] = 0.0;
    // e_n = exp(-j 2 pi n theta): exact phase reduction every ACT_ANCHOR-th
    // sample of a thread, rotations by exp(-j 2 pi ACT_NT theta) in between
    // (a few ulp from the exact value, against one sincospi per sample)
    const cd rot = cconj(cis2pi(frac_mul((double)ACT_NT, th)));
    cd e{1.0, 0.0};
    int it = 0;
    if (full) {
      for (int n = tid; n < N; n += ACT_NT, ++it) {
        const double dn = (double)n;
        e = (it % ACT_ANCHOR == 0) ? cconj(cis2pi(frac_mul(dn, th))) : cmul(e, rot);
        const cd we = cmul(wb[n], e);
        const cd re = cmul(rb[n], e);
        const double x = dn - cN;
        acc[0] += we.x; acc[1] += we.y;
        acc[2] = fma(dn, we.x, acc[2]); acc[3] = fma(dn, we.y, acc[3]);
        const double d2 = dn * dn;
        acc[4] = fma(d2, we.x, acc[4]); acc[5] = fma(d2, we.y, acc[5]);
        acc[6] += re.x; acc[7] += re.y;
        acc[8] = fma(x, re.x, acc[8]); acc[9] = fma(x, re.y, acc[9]);
        const double x2 = x * x;
        acc[10] = fma(x2, re.x, acc[10]); acc[11] = fma(x2, re.y, acc[11]);
        const double x3 = x2 * x;
        acc[12] = fma(x3, re.x, acc[12]); acc[13] = fma(x3, re.y, acc[13]);
      }
    } else {
      for (int n = tid; n < N; n += ACT_NT, ++it) {
        const double dn = (double)n;
        e = (it % ACT_ANCHOR == 0) ? cconj(cis2pi(frac_mul(dn, th))) : cmul(e, rot);
        const cd we = cmul(wb[n], e);
        const cd re = cmul(rb[n], e);
        const double x = dn - cN;
        acc[0] += we.x; acc[1] += we.y;
        acc[6] += re.x; acc[7] += re.y;
        acc[8] = fma(x, re.x, acc[8]); acc[9] = fma(x, re.y, acc[9]);
      }
    }
    block_sum<ACT_NT, 14>(acc, red);
    if (tid == 0)
      active_out(acc, full, in, j, nk, 1.0 / delta[in.off + N - 1], coef[bi], oq, orr, ou, os, ot,
                 ov, ox, cq, cs);
    __syncthreads();
    // further observation vectors: q (and r, u at active points) with the same phases
    for (int gv = 1; gv < vv.G; ++gv) {
      const cd* wg = w + gv * vv.wstride + in.off;
      double a6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      int it2 = 0;
      for (int n = tid; n < N; n += ACT_NT, ++it2) {
        const double dn = (double)n;
        e = (it2 % ACT_ANCHOR == 0) ? cconj(cis2pi(frac_mul(dn, th))) : cmul(e, rot);
        const cd we = cmul(wg[n], e);
        a6[0] += we.x; a6[1] += we.y;
        if (full) {
          a6[2] = fma(dn, we.x, a6[2]); a6[3] = fma(dn, we.y, a6[3]);
          const double d2 = dn * dn;
          a6[4] = fma(d2, we.x, a6[4]); a6[5] = fma(d2, we.y, a6[5]);
        }
      }
      block_sum<ACT_NT, 6>(a6, red);
      if (tid == 0) vec_out(a6, full, in, j, nk, gv, vv, oq, orr, ou, cq);
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// The same sums, one workgroup per instance of at most ACT_LDS_N samples: w
// and rho are read from HBM once into LDS, and each wave takes points j =
// wave, wave + 4, ..., its lanes striding over the samples with the phase
// rotated by exp(-j 2 pi 64 theta) between exact evaluations every
// ACT_ANCHOR_W samples, and wave reductions (same bits in every lane).  The
// item-parallel k_active instead reads both vectors once per point.
// ---------------------------------------------------------------------------
constexpr int ACTL_NT = 1024;
constexpr int ACT_ANCHOR_W = 8;

__global__ __launch_bounds__(ACTL_NT) void k_active_lds(const InstInfo* __restrict__ info,
                                                        const int32_t* __restrict__ req,
                                                        const int32_t* __restrict__ Keval,
                                                        const int32_t* __restrict__ ncand,
                                                        int nmode, const double* __restrict__ theta,
                                                        const int32_t* __restrict__ cand,
                                                        const cd* __restrict__ w,
                                                        const cd* __restrict__ rho,
                                                        const double* __restrict__ delta,
                                                        const SepCoef* __restrict__ coef,
                                                        cd* __restrict__ oq, cd* __restrict__ orr,
                                                        cd* __restrict__ ou, cd* __restrict__ os,
                                                        cd* __restrict__ ot, cd* __restrict__ ov,
                                                        cd* __restrict__ ox, cd* __restrict__ cq,
                                                        double* __restrict__ cs, Vecs vv,
                                                        const int32_t* __restrict__ order) {
  const int bi = order ? order[blockIdx.x] : blockIdx.x;
  const int32_t rq = req ? req[bi] : REQ_EVAL;
  const InstInfo in = info[bi];
  const int nk = (rq & REQ_EVAL) ? Keval[bi] : 0;
  const int nc = ((rq & REQ_GRID) && ncand) ? ncand[bi] : 0;
  const int npts = nk + nc;
  const int N = in.N;
  if (!use_lds_active(nmode, N, in.P, npts)) return;
  extern __shared__ cd actl_sh[];
  cd* sw = actl_sh;      // [N]
  cd* sr = actl_sh + N;  // [N]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  batched_for<8>(tid, ACTL_NT, N, [&](int t) { return cd2{w[in.off + t], rho[in.off + t]}; },
                 [&](int t, cd2 v) {
    sw[t] = v.a;
    sr[t] = v.b;
  });
  __syncthreads();
  const double cN = 0.5 * (double)(N - 1);
  const double idl = 1.0 / delta[in.off + N - 1];
  const SepCoef& cf = coef[bi];
  for (int j = wv; j < npts; j += ACTL_NT / 64) {
    const bool full = j < nk;
    const double th = full ? theta[in.koff + j] : (double)cand[in.coff + (j - nk)] / (double)in.L;
    const cd rot = cconj(cis2pi(frac_mul(64.0, th)));
    double acc[14];
#pragma unroll
    for (int i = 0; i < 14; ++i) acc[i] = 0.0;
    cd e{1.0, 0.0};
    int it = 0;
    for (int n = lane; n < N; n += 64, ++it) {
      const double dn = (double)n;
      e = (it % ACT_ANCHOR_W == 0) ? cconj(cis2pi(frac_mul(dn, th))) : cmul(e, rot);
      const cd we = cmul(sw[n], e);
      const cd re = cmul(sr[n], e);
      const double x = dn - cN;
      acc[0] += we.x; acc[1] += we.y;
      acc[6] += re.x; acc[7] += re.y;
      acc[8] = fma(x, re.x, acc[8]); acc[9] = fma(x, re.y, acc[9]);
      if (full) {
        acc[2] = fma(dn, we.x, acc[2]); acc[3] = fma(dn, we.y, acc[3]);
        const double d2 = dn * dn;
        acc[4] = fma(d2, we.x, acc[4]); acc[5] = fma(d2, we.y, acc[5]);
        const double x2 = x * x;
        acc[10] = fma(x2, re.x, acc[10]); acc[11] = fma(x2, re.y, acc[11]);
        const double x3 = x2 * x;
        acc[12] = fma(x3, re.x, acc[12]); acc[13] = fma(x3, re.y, acc[13]);
      }
    }
#pragma unroll
    for (int i = 0; i < 14; ++i) acc[i] = wave_sum(acc[i]);
    if (lane == 0) active_out(acc, full, in, j, nk, idl, cf, oq, orr, ou, os, ot, ov, ox, cq, cs);
  }
  // further observation vectors: w_g replaces w in LDS; q (and r, u at active
  // points) with the same phases
  for (int gv = 1; gv < vv.G; ++gv) {
    __syncthreads();
    for (int t = tid; t < N; t += ACTL_NT) sw[t] = w[gv * vv.wstride + in.off + t];
    __syncthreads();
    for (int j = wv; j < npts; j += ACTL_NT / 64) {
      const bool full = j < nk;
      const double th = full ? theta[in.koff + j] : (double)cand[in.coff + (j - nk)] / (double)in.L;
      const cd rot = cconj(cis2pi(frac_mul(64.0, th)));
      double a6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      cd e{1.0, 0.0};
      int it = 0;
      for (int n = lane; n < N; n += 64, ++it) {
        const double dn = (double)n;
        e = (it % ACT_ANCHOR_W == 0) ? cconj(cis2pi(frac_mul(dn, th))) : cmul(e, rot);
        const cd we = cmul(sw[n], e);
        a6[0] += we.x; a6[1] += we.y;
        if (full) {
          a6[2] = fma(dn, we.x, a6[2]); a6[3] = fma(dn, we.y, a6[3]);
          const double d2 = dn * dn;
          a6[4] = fma(d2, we.x, a6[4]); a6[5] = fma(d2, we.y, a6[5]);
        }
      }
#pragma unroll
      for (int i = 0; i < 6; ++i) a6[i] = wave_sum(a6[i]);
      if (lane == 0) vec_out(a6, full, in, j, nk, gv, vv, oq, orr, ou, cq);
    }
  }
}

// ---------------------------------------------------------------------------
// The same quantities by the non-uniform FFT (Sec. III-B/C use the NUFFT for
// these off-grid Fourier sums), one workgroup per instance.  Gaussian gridding
// (Greengard and Lee): with centred modes m = n - h (h = N/2), an oversampled
// grid of P >= 2N points (grid spacing 2 pi / P) and the Gaussian
// g(t) = exp(-t^2 / (4 tau)), whose Fourier transform is
// sqrt(4 pi tau) exp(-m^2 tau),
//   sum_n x_n e^{-j 2 pi n theta}
//     = e^{-j 2 pi h theta} sum_m [x_{m+h} / ghat(m)] e^{-j m omega}    (omega = 2 pi theta)
//     ~ e^{-j 2 pi h theta} (2 pi / P) sum_l g(omega - 2 pi l / P) X_l,
// X = FFT_P of the deconvolved sequence, the sum over the 2 NU_MSP grid points
// nearest to theta, and tau = pi NU_MSP / (N^2 R (R - 1/2)) with R = P / N.
// The Gaussian's argument is formed as (2 pi / P)(theta P - l) (theta P is
// exact for P a power of two) and the phase e^{-j 2 pi h theta} from the
// reduced fraction of h theta, so no rounding grows with N.  The seven
// sequences w, n w, n^2 w, x^a rho (a = 0..3) are transformed one at a time
// in LDS (or, for P > CONV_LDS_P, in the instance's scratch after its four P
// blocks); G_a at the points wait in scratch blocks 1-3.  Block 0 keeps the
// spectrum of rho that the Gohberg-Semencul apply left there: a later round
// that only evaluates the grid reuses it for omega.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NU_NT) void k_active_nufft(const InstInfo* __restrict__ info,
                                                        const int32_t* __restrict__ req,
                                                        const int32_t* __restrict__ Keval,
                                                        const int32_t* __restrict__ ncand,
                                                        int nmode, const double* __restrict__ theta,
                                                        const int32_t* __restrict__ cand,
                                                        const cd* __restrict__ w,
                                                        const cd* __restrict__ rho,
                                                        const double* __restrict__ delta,
                                                        const SepCoef* __restrict__ coef,
                                                        const cd* __restrict__ tws,
                                                        cd* __restrict__ scratch,
                                                        cd* __restrict__ oq, cd* __restrict__ orr,
                                                        cd* __restrict__ ou, cd* __restrict__ os,
                                                        cd* __restrict__ ot, cd* __restrict__ ov,
                                                        cd* __restrict__ ox, cd* __restrict__ cq,
                                                        double* __restrict__ cs,
                                                        const int32_t* __restrict__ order) {
  const int bi = order ? order[blockIdx.x] : blockIdx.x;
  const int32_t rq = req ? req[bi] : REQ_EVAL;
  const InstInfo in = info[bi];
  const int nk = (rq & REQ_EVAL) ? Keval[bi] : 0;
  const int nc = ((rq & REQ_GRID) && ncand) ? ncand[bi] : 0;
  const int npts = nk + nc;
  const int N = in.N, P = in.P, logP = in.logP;
  if (!use_nufft(nmode, N, P, npts)) return;
  extern __shared__ cd lds_sh[];
  __shared__ cd s_tw[FFT_TWL];
  __shared__ double s_e3[2 * NU_MSP];
  const int tid = threadIdx.x;
  const double TWO_PI = 6.283185307179586476925286766559;
  const double R = (double)P / (double)N;
  const double tau = 3.14159265358979323846 * NU_MSP / ((double)N * (double)N * R * (R - 0.5));
  const double ag = (TWO_PI / P) * (TWO_PI / P) / (4.0 * tau);  // g at grid offset u: exp(-ag u^2)
  const double sq = sqrt(4.0 * 3.14159265358979323846 * tau);
  const int h = N / 2;
  const double cN = 0.5 * (double)(N - 1);
  load_tw_head<NU_NT>(s_tw, tws);
  // exp(-ag t^2) for the offsets t = -(NU_MSP-1) .. NU_MSP
  if (tid < 2 * NU_MSP) {
    const double t = (double)(tid - (NU_MSP - 1));
    s_e3[tid] = exp(-ag * t * t);
  }
  const cd* wb = w + in.off;
  const cd* rb = rho + in.off;
  cd* Gs = scratch + in.poff + P;  // G_a at the points: Gs[a * npts + p]
  auto point = [&](int p) {
    return p < nk ? theta[in.koff + p] : (double)cand[in.coff + (p - nk)] / (double)in.L;
  };
  auto body = [&](cd* __restrict__ buf) __attribute__((always_inline)) {
    for (int j = 0; j < 7; ++j) {
      const bool all = (j == 0 || j == 3 || j == 4);  // also needed at the candidates
      const int np = all ? npts : nk;
      if (np == 0) continue;
      // deconvolved sequence on centred modes: buf[m mod P] = x_{m+h} / ghat(m)
      batched_for<4>(tid, NU_NT, P, [&](int t) {
        const int m = t < N - h ? t : t - P;  // centred mode stored at t
        cd v{0.0, 0.0};
        if (m >= -h && m < N - h) {
          const int n = m + h;
          const double dn = (double)n, x = dn - cN;
          const cd src = j < 3 ? wb[n] : rb[n];
          const double wgt = j == 0 ? 1.0 : j == 1 ? dn : j == 2 ? dn * dn
                           : j == 3 ? 1.0 : j == 4 ? x : j == 5 ? x * x : x * x * x;
          v = cscale(src, wgt * exp((double)m * (double)m * tau) / sq);
        }
        return v;
      }, [&](int t, cd v) { buf[pidx(t)] = v; });
      __syncthreads();
      dif_fftn<NU_NT>(buf, buf, 1, logP, false, false, s_tw, tws);
      // interpolation at the points (spectrum in bit-reversed order)
      for (int p = tid; p < np; p += NU_NT) {
        const double th = point(p);
        const double sP = th * (double)P;  // exact: P is a power of two
        const double fl = floor(sP);
        const double d = sP - fl;          // exact
        const int l0 = (int)fl;
        // exp(-ag (d - t)^2) = exp(-ag d^2) exp(2 ag d t) exp(-ag t^2)
        const double e1 = exp(-ag * d * d);
        const double e2 = exp(2.0 * ag * d);
        double e2t = exp(-2.0 * ag * d * (double)(NU_MSP - 1));  // e2^t at t = -(NU_MSP-1)
        cd acc{0.0, 0.0};
#pragma unroll 4
        for (int i = 0; i < 2 * NU_MSP; ++i) {
          const int l = (l0 + i - (NU_MSP - 1)) & (P - 1);
          const double g = e1 * e2t * s_e3[i];
          const cd X = buf[pidx(bitrev(l, logP))];
          acc.x = fma(g, X.x, acc.x);
          acc.y = fma(g, X.y, acc.y);
          e2t *= e2;
        }
        const cd ph = cconj(cis2pi(frac_mul((double)h, th)));
        cd val = cscale(cmul(acc, ph), TWO_PI / P);
        if (j == 1) val = cscale(val, TWO_PI);
        if (j == 2) val = cscale(val, TWO_PI * TWO_PI);
        if (j == 0) {
          if (p < nk) oq[in.koff + p] = val; else cq[in.coff + (p - nk)] = val;
        } else if (j == 1) {
          orr[in.koff + p] = val;
        } else if (j == 2) {
          ou[in.koff + p] = val;
        } else {
          Gs[(int64_t)(j - 3) * npts + p] = val;
        }
      }
      __syncthreads();
    }
  };
  if (P > CONV_LDS_P) body(scratch + in.poff + 4 * (int64_t)P);
  else body(lds_sh);
  // s, t, v, x from the G_a as in the direct form
  const double idl = 1.0 / delta[in.off + N - 1];
  const SepCoef& cf = coef[bi];
  for (int p = tid; p < npts; p += NU_NT) {
    const bool full = p < nk;
    cd G[4];
    for (int a = 0; a < 4; ++a)
      G[a] = (full || a < 2) ? Gs[(int64_t)a * npts + p] : cd{0.0, 0.0};
    const int nq = full ? 4 : 1;
    cd outv[4];
    for (int qk = 0; qk < nq; ++qk) {
      const double* C = cf.c[qk];
      const int am = (qk == 0) ? 1 : 3;
      cd a2{0.0, 0.0};
      for (int a = 0; a <= am; ++a)
        for (int b2 = 0; b2 <= am; ++b2) {
          const double cab = C[a * 4 + b2];
          if (cab != 0.0) {
            const cd pr = cmulc(G[a], G[b2]);
            a2.x = fma(cab, pr.x, a2.x);
            a2.y = fma(cab, pr.y, a2.y);
          }
        }
      outv[qk] = cscale(a2, idl);
    }
    if (full) {
      const int64_t o = in.koff + p;
      os[o] = cd{outv[0].x, 0.0};
      ot[o] = outv[1];
      ov[o] = outv[2];
      ox[o] = outv[3];
    } else {
      cs[in.coff + (p - nk)] = outv[0].x;
    }
  }
}

hipError_t launch_active(const InstInfo* info, const int32_t* req, const int32_t* Keval,
                         const int32_t* ncand, int32_t* prefix, int B, const double* theta,
                         const int32_t* cand, const cd* w, const cd* rho, const double* delta,
                         const SepCoef* coef, cd* oq, cd* orr, cd* ou, cd* os, cd* ot, cd* ov,
                         cd* ox, cd* cq, double* cs, int nblocks, int nmode, const cd* tws,
                         cd* scratch, int maxP, hipStream_t st, Vecs vv, const int32_t* order) {
  if (!scratch) nmode = 1;  // no scratch for the NUFFT form: direct sums only
  if (vv.G > 1) nmode = 1;  // several observation vectors: direct sums
  // every instance has N <= P/2; with P <= 2 ACT_LDS_N throughout, the direct
  // sums all run in k_active_lds and the item-parallel pair has nothing to do
  if (maxP > 2 * ACT_LDS_N) {
    hipLaunchKernelGGL(k_item_scan, dim3(1), dim3(1024), 0, st, info, req, Keval, ncand, B, nmode,
                       prefix);
    hipLaunchKernelGGL(k_active, dim3(nblocks), dim3(ACT_NT), 0, st, info, req, Keval, prefix, B,
                       theta, cand, w, rho, delta, coef, oq, orr, ou, os, ot, ov, ox, cq, cs, vv);
  }
  {
    // N <= P/2 for every instance, so 2 * min(P, 2 ACT_LDS_N) / 2 points cover w and rho
    const int pl = maxP < 2 * ACT_LDS_N ? maxP : 2 * ACT_LDS_N;
    const size_t shm = (size_t)pl * sizeof(cd);
    (void)hipFuncSetAttribute((const void*)k_active_lds,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    hipLaunchKernelGGL(k_active_lds, dim3(B), dim3(ACTL_NT), shm, st, info, req, Keval, ncand,
                       nmode, theta, cand, w, rho, delta, coef, oq, orr, ou, os, ot, ov, ox, cq,
                       cs, vv, order);
  }
  if (nmode != 1) {
    const size_t shm = (size_t)padded(maxP < CONV_LDS_P ? maxP : CONV_LDS_P) * sizeof(cd);
    (void)hipFuncSetAttribute((const void*)k_active_nufft,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    hipLaunchKernelGGL(k_active_nufft, dim3(B), dim3(NU_NT), shm, st, info, req, Keval, ncand,
                       nmode, theta, cand, w, rho, delta, coef, tws, scratch, oq, orr, ou, os, ot,
                       ov, ox, cq, cs, order);
  }
  return hipGetLastError();
}

}  // namespace sfls
