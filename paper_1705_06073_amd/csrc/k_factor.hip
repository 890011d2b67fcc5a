// a1: covariance generator c;  a2: Levinson-Durbin factorisation into the
// Gohberg-Semencul generator (rho, delta).
#include "sfls_kernels.hpp"
#include "k_launch.hpp"

namespace sfls {

// ---------------------------------------------------------------------------
// a1.  c_i = beta [i = 0] + sum_k gamma_k exp(j 2 pi i theta_k)  (eq. py, first
// column).  Grid: (tiles of TC_SPT * 256 samples, instances); thread t takes
// samples i0 + 256 s (s < TC_SPT) of its tile.  theta/gamma of the instance
// are staged through LDS in chunks of 256 together with the rotation
// exp(j 2 pi 256 theta_k), so that a thread evaluates one exact phase per
// component (exact reduction of i0 theta mod 1) and rotates it to its other
// samples (a few ulp from the exact phases).
// ---------------------------------------------------------------------------
constexpr int TC_SPT = 4;

__global__ __launch_bounds__(256) void k_toeplitz_column(const InstInfo* __restrict__ info,
                                                         const int32_t* __restrict__ req,
                                                         const int32_t* __restrict__ Kcnt,
                                                         const double* __restrict__ theta,
                                                         const double* __restrict__ gamma,
                                                         const double* __restrict__ beta,
                                                         cd* __restrict__ c, int nmode) {
  const int b = blockIdx.y;
  if (req && !(req[b] & REQ_EVAL)) return;
  const InstInfo in = info[b];
  const int tile = blockIdx.x * 256 * TC_SPT;
  if (tile >= in.N) return;
  const int K = Kcnt[b];
  if (use_nufft_col(nmode, in.N, in.P, K)) return;  // k_toeplitz_nufft writes it
  __shared__ double sth[256], sga[256];
  __shared__ cd srot[256];
  const int i0 = tile + threadIdx.x;
  cd acc[TC_SPT];
#pragma unroll
  for (int s = 0; s < TC_SPT; ++s) acc[s] = cd{0.0, 0.0};
  const double di = (double)i0;
  for (int k0 = 0; k0 < K; k0 += 256) {
    __syncthreads();
    if (k0 + threadIdx.x < K) {
      const double th = theta[in.koff + k0 + threadIdx.x];
      sth[threadIdx.x] = th;
      sga[threadIdx.x] = gamma[in.koff + k0 + threadIdx.x];
      srot[threadIdx.x] = cis2pi(frac_mul(256.0, th));
    }
    __syncthreads();
    const int kn = min(256, K - k0);
    for (int k = 0; k < kn; ++k) {
      cd e = cis2pi(frac_mul(di, sth[k]));
      const cd r = srot[k];
      const double g = sga[k];
#pragma unroll
      for (int s = 0; s < TC_SPT; ++s) {
        if (s > 0) e = cmul(e, r);
        acc[s].x = fma(g, e.x, acc[s].x);
        acc[s].y = fma(g, e.y, acc[s].y);
      }
    }
  }
#pragma unroll
  for (int s = 0; s < TC_SPT; ++s) {
    const int i = i0 + 256 * s;
    if (i < in.N) {
      cd v = acc[s];
      if (i == 0) { v.x += beta[b]; v.y = 0.0; }
      c[in.off + i] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// a1 by the type-1 non-uniform FFT (Gaussian gridding, Greengard and Lee; the
// paper evaluates products with Psi by NUFFT, Sec. III-B).  With centred
// modes m = i - h (h = N/2), gamma'_k = gamma_k e^{j 2 pi h theta_k} and the
// Gaussian g(x) = exp(-x^2 / (4 tau)), whose transform is
// sqrt(4 pi tau) exp(-m^2 tau),
//   c_{m+h} - beta [m+h = 0] = sum_k gamma'_k e^{j m omega_k}
//     ~ e^{m^2 tau} / sqrt(4 pi tau) (2 pi / P) sum_l H_l e^{+j 2 pi m l / P},
//   H_l = sum_k gamma'_k g(2 pi l / P - omega_k)   (periodic, 2 NU_MSP points),
// on the oversampled grid of P >= 2N points with the tau of the type-2 form.
// The spreading is a gather: the frequencies' grid positions are sorted in
// LDS (a frequency within NU_MSP points of either end also enters shifted by
// P), so each grid point adds its neighbours in a fixed order and the column
// does not depend on scheduling.  One workgroup per instance; the transform
// runs in the instance's scratch buffer after its four P blocks (P >
// CONV_LDS_P), which an evaluation round has not yet used when this runs.
// ---------------------------------------------------------------------------
constexpr int NUC_NT = 512;

__device__ __forceinline__ int lower_bound_i64(const int64_t* a, int n, int64_t v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(NUC_NT) void k_toeplitz_nufft(const InstInfo* __restrict__ info,
                                                           const int32_t* __restrict__ req,
                                                           const int32_t* __restrict__ Kcnt,
                                                           const double* __restrict__ theta,
                                                           const double* __restrict__ gamma,
                                                           const double* __restrict__ beta,
                                                           const cd* __restrict__ tws,
                                                           cd* __restrict__ scratch,
                                                           cd* __restrict__ c, int nmode) {
  const int b = blockIdx.x;
  if (req && !(req[b] & REQ_EVAL)) return;
  const InstInfo in = info[b];
  const int K = Kcnt[b];
  const int N = in.N, P = in.P, logP = in.logP;
  if (!use_nufft_col(nmode, N, P, K)) return;
  extern __shared__ int64_t nuc_sh[];
  int64_t* s_key = nuc_sh;                                        // [2 NUC_KMAX]
  double* s_d = reinterpret_cast<double*>(nuc_sh + 2 * NUC_KMAX);  // [NUC_KMAX]
  cd* s_g = reinterpret_cast<cd*>(s_d + NUC_KMAX);                 // [NUC_KMAX]
  __shared__ cd s_tw[FFT_TWL];
  const int tid = threadIdx.x;
  const double TWO_PI = 6.283185307179586476925286766559;
  const double R = (double)P / (double)N;
  const double tau = 3.14159265358979323846 * NU_MSP / ((double)N * (double)N * R * (R - 0.5));
  const double ag = (TWO_PI / P) * (TWO_PI / P) / (4.0 * tau);
  const double sq = sqrt(4.0 * 3.14159265358979323846 * tau);
  const int h = N / 2;
  load_tw_head<NUC_NT>(s_tw, tws);
  // grid positions: key = (floor(theta P) + P [+- P]) << 32 | k, unique per entry
  int E = 2;
  while (E < 2 * K) E <<= 1;
  for (int k = tid; k < K; k += NUC_NT) {
    const double th = theta[in.koff + k];
    const double sP = th * (double)P;  // exact: P is a power of two
    const double fl = floor(sP);
    int l0 = (int)fl;
    const double d = sP - fl;          // exact
    l0 = l0 < 0 ? 0 : (l0 > P - 1 ? P - 1 : l0);
    s_d[k] = d;
    s_g[k] = cscale(cis2pi(frac_mul((double)h, th)), gamma[in.koff + k]);
    s_key[2 * k] = ((int64_t)(l0 + P) << 32) | (int64_t)k;
    int64_t dup = INT64_MAX;
    if (l0 < NU_MSP) dup = ((int64_t)(l0 + 2 * P) << 32) | (int64_t)k;
    else if (l0 >= P - NU_MSP) dup = ((int64_t)l0 << 32) | (int64_t)k;
    s_key[2 * k + 1] = dup;
  }
  for (int i = 2 * K + tid; i < E; i += NUC_NT) s_key[i] = INT64_MAX;
  __syncthreads();
  // bitonic sort, ascending
  for (int kk = 2; kk <= E; kk <<= 1) {
    for (int j = kk >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < E; i += NUC_NT) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const int64_t a = s_key[i], bb = s_key[ixj];
          const bool up = (i & kk) == 0;
          if ((a > bb) == up) {
            s_key[i] = bb;
            s_key[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  // spreading by gather, one grid point per thread and tile
  cd* buf = scratch + in.poff + 4 * (int64_t)P;
  for (int l0 = 0; l0 < P; l0 += NUC_NT) {
    const int l = l0 + tid;
    const int lo = lower_bound_i64(s_key, E, (int64_t)(l0 - NU_MSP + P) << 32);
    const int hi = lower_bound_i64(s_key, E, (int64_t)(l0 + NUC_NT + NU_MSP - 1 + P) << 32);
    cd acc{0.0, 0.0};
    for (int j = lo; j < hi; ++j) {
      const int64_t key = s_key[j];
      const int t = l - ((int)(key >> 32) - P);
      if (t >= -(NU_MSP - 1) && t <= NU_MSP) {
        const int k = (int)(key & 0xffffffff);
        const double x = (double)t - s_d[k];
        const double g = exp(-ag * x * x);
        acc.x = fma(g, s_g[k].x, acc.x);
        acc.y = fma(g, s_g[k].y, acc.y);
      }
    }
    buf[pidx(l)] = acc;
  }
  __syncthreads();
  dif_fftn<NUC_NT>(buf, buf, 1, logP, true, false, s_tw, tws);  // kernel e^{+j}, bit-reversed out
  const double sc = TWO_PI / (double)P / sq;
  for (int i = tid; i < N; i += NUC_NT) {
    const int m = i - h;
    const cd X = buf[pidx(bitrev(m & (P - 1), logP))];
    cd v = cscale(X, exp((double)m * (double)m * tau) * sc);
    if (i == 0) { v.x += beta[b]; v.y = 0.0; }
    c[in.off + i] = v;
  }
}

// ---------------------------------------------------------------------------
// a2.  Levinson-Durbin in the forward/backward predictor form.
//
//   a^(0) = [1], b^(0) = [1], delta_0 = c_0
//   step n = 1..N-1:
//     eps_n   = sum_{j<n} c_{j+1} conj(b_j)          (= sum_i c_{n-i} a_i)
//     k_n     = -eps_n / delta_{n-1}
//     a_j    <- a_j + k_n b_{j-1}
//     b_j    <- b_{j-1} + conj(k_n) a_j              (b_j = conj(a_{n-j}))
//     delta_n = delta_{n-1} (1 - |k_n|^2)
//   rho = b^(N-1)  (rho_i = conj(a_{N-1-i}), so rho_{N-1} = 1)
//
// a, b and c_{j+1} stay in registers: element j lives in slot j / T of thread
// j % T.  The only data movement per step is the shift b_{j-1} -> j, done
// with a DPP wave_shr:1 inside each wave and an LDS hand-off of lane 63 across
// waves (and from the last wave into the next slot).  The dot product for the
// next step is fused into the update pass; one barrier per step carries both
// the wave partial sums and the hand-off values (double-buffered by parity).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double shr1_f64(double v, double old) {
  int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), 0x138, 0xF, 0xF, false);
  int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), 0x138, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

template <int T, int S>
__global__ __launch_bounds__(T) void k_levinson(const InstInfo* __restrict__ info,
                                                const int32_t* __restrict__ req,
                                                const cd* __restrict__ c, cd* __restrict__ rho,
                                                double* __restrict__ delta_out,
                                                double* __restrict__ logdet,
                                                int32_t* __restrict__ status,
                                                int64_t* __restrict__ failed) {
  constexpr int W = T / 64;
  const int bi = blockIdx.x;
  if (req && !(req[bi] & REQ_EVAL)) return;
  const InstInfo in = info[bi];
  const int N = in.N;
  if (N > T * S) return;  // host dispatch guarantees N <= T*S
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;

  __shared__ cd xb[2][W][S];
  __shared__ cd xp[2][W];
  __shared__ double dl[T * S];
  __shared__ double red[W];

  const cd* cb = c + in.off;
  cd a[S], bb[S], cc[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int j = s * T + tid;
    a[s] = cd{j == 0 ? 1.0 : 0.0, 0.0};
    bb[s] = a[s];
    cc[s] = (j + 1 < N) ? cb[j + 1] : cd{0.0, 0.0};
  }
  for (int e = tid; e < 2 * W * S; e += T) (&xb[0][0][0])[e] = cd{0.0, 0.0};
  double dlt = cb[0].x;
  int fail = (dlt > 0.0 && isfinite(dlt)) ? -1 : 0;
  if (tid == 0) dl[0] = dlt;
  cd eps = (N > 1) ? cb[1] : cd{0.0, 0.0};
  __syncthreads();

  double inv = 1.0 / dlt;
  int n = 1;
  for (; n < N && fail < 0; ++n) {
    const int par = n & 1, ppar = par ^ 1;
    const cd k{-eps.x * inv, -eps.y * inv};
    const double dn = dlt * (1.0 - cabs2(k));
    if (!(dn > 0.0) || !isfinite(dn)) { fail = n; break; }
    // reciprocal for the next step, off the critical path of this one
    const double inv_next = 1.0 / dn;
    // hand-off values from the neighbouring wave (read for every slot at once)
    cd inc[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if (wv > 0) inc[s] = xb[ppar][wv - 1][s];
      else inc[s] = (s > 0) ? xb[ppar][W - 1][s - 1] : cd{0.0, 0.0};
    }
    cd part[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      part[s] = cd{0.0, 0.0};
      if (s * T <= n) {
        cd sh{shr1_f64(bb[s].x, inc[s].x), shr1_f64(bb[s].y, inc[s].y)};
        const cd ao = a[s];
        a[s] = cfma(k, sh, ao);                 // a_j + k b_{j-1}
        bb[s] = cfmac(ao, k, sh);               // b_{j-1} + conj(k) a_j
        part[s] = cmulc(cc[s], bb[s]);          // c_{j+1} conj(b_j)
      }
    }
    if (lane == 63) {
#pragma unroll
      for (int s = 0; s < S; ++s)
        if (s * T <= n) xb[par][wv][s] = bb[s];
    }
    // pairwise sum of the slot partials, then across the wave
#pragma unroll
    for (int w2 = 1; w2 < S; w2 <<= 1)
#pragma unroll
      for (int s = 0; s + w2 < S; s += 2 * w2) part[s] = cadd(part[s], part[s + w2]);
    const cd acc = wave_sum(part[0]);
    if (lane == 0) xp[par][wv] = acc;
    if (tid == 0) dl[n] = dn;
    __syncthreads();
    cd e{0.0, 0.0};
#pragma unroll
    for (int w = 0; w < W; ++w) e = cadd(e, xp[par][w]);
    eps = e;
    dlt = dn;
    inv = inv_next;
  }
  __syncthreads();

  // outputs: rho = b, delta, ln|C|
  cd* rb = rho + in.off;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int j = s * T + tid;
    if (j < N) rb[j] = bb[s];
  }
  double part = 0.0;
  const int nvalid = (fail < 0) ? N : fail;
  for (int j = tid; j < nvalid; j += T) {
    part += log(dl[j]);
    if (delta_out) delta_out[in.off + j] = dl[j];
  }
  part = wave_sum(part);
  if (lane == 0) red[wv] = part;
  __syncthreads();
  if (tid == 0) {
    double ld = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) ld += red[w];
    if (logdet) logdet[bi] = (fail < 0) ? ld : __builtin_nan("");
    if (status) status[bi] = (fail < 0) ? 0 : -4;
    if (failed) failed[bi] = fail;
  }
}

#define LEV_INST(T, S) template __global__ void k_levinson<T, S>(const InstInfo*, const int32_t*, \
    const cd*, cd*, double*, double*, int32_t*, int64_t*);

// Host-side dispatch: one workgroup per instance; the slot count is chosen
// from the largest N of the batch.
hipError_t launch_toeplitz_column(const InstInfo* info, const int32_t* req, const int32_t* Kcnt,
                                  const double* theta, const double* gamma, const double* beta,
                                  cd* c, int B, int maxN, hipStream_t st, int nmode,
                                  const cd* tws, cd* scratch, int maxP) {
  if (!scratch || !tws || maxP <= CONV_LDS_P) nmode = 1;  // no room for the transform: direct
  dim3 grid((maxN + 256 * TC_SPT - 1) / (256 * TC_SPT), B);
  hipLaunchKernelGGL(k_toeplitz_column, grid, dim3(256), 0, st, info, req, Kcnt, theta, gamma,
                     beta, c, nmode);
  if (nmode != 1) {
    const size_t shm = (size_t)NUC_KMAX * (2 * sizeof(int64_t) + sizeof(double) + sizeof(cd));
    (void)hipFuncSetAttribute((const void*)k_toeplitz_nufft,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    hipLaunchKernelGGL(k_toeplitz_nufft, dim3(B), dim3(NUC_NT), shm, st, info, req, Kcnt, theta,
                       gamma, beta, tws, scratch, c, nmode);
  }
  return hipGetLastError();
}

hipError_t launch_levinson(const InstInfo* info, const int32_t* req, const cd* c, cd* rho,
                           double* delta, double* logdet, int32_t* status, int64_t* failed, int B,
                           int maxN, hipStream_t st) {
#define LEV_GO(T, S)                                                                      \
  hipLaunchKernelGGL((k_levinson<T, S>), dim3(B), dim3(T), 0, st, info, req, c, rho, delta, \
                     logdet, status, failed);                                             \
  return hipGetLastError();
  if (maxN <= 64) { LEV_GO(64, 1) }
  if (maxN <= 128) { LEV_GO(64, 2) }
  if (maxN <= 256) { LEV_GO(64, 4) }
  if (maxN <= 512) { LEV_GO(128, 4) }
  if (maxN <= 1024) { LEV_GO(256, 4) }
  if (maxN <= 2048) { LEV_GO(256, 8) }
  if (maxN <= 4096) { LEV_GO(512, 8) }
#undef LEV_GO
  return hipErrorInvalidValue;
}

}  // namespace sfls
