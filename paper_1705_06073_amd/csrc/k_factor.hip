// a1: covariance generator c;  a2: Levinson-Durbin factorisation into the
// Gohberg-Semencul generator (rho, delta).
#include "sfls_kernels.hpp"
#include "k_launch.hpp"

namespace sfls {

// ---------------------------------------------------------------------------
// a1.  c_i = beta [i = 0] + sum_k gamma_k exp(j 2 pi i theta_k)  (eq. py, first
// column).  Grid: (tiles of 256 samples, instances).  theta/gamma of the
// instance are staged through LDS in chunks of 256.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_toeplitz_column(const InstInfo* __restrict__ info,
                                                         const int32_t* __restrict__ req,
                                                         const int32_t* __restrict__ Kcnt,
                                                         const double* __restrict__ theta,
                                                         const double* __restrict__ gamma,
                                                         const double* __restrict__ beta,
                                                         cd* __restrict__ c) {
  const int b = blockIdx.y;
  if (req && !(req[b] & REQ_EVAL)) return;
  const InstInfo in = info[b];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (blockIdx.x * 256 >= in.N) return;
  const int K = Kcnt[b];
  __shared__ double sth[256], sga[256];
  cd acc{0.0, 0.0};
  const double di = (double)i;
  for (int k0 = 0; k0 < K; k0 += 256) {
    __syncthreads();
    if (k0 + threadIdx.x < K) {
      sth[threadIdx.x] = theta[in.koff + k0 + threadIdx.x];
      sga[threadIdx.x] = gamma[in.koff + k0 + threadIdx.x];
    }
    __syncthreads();
    const int kn = min(256, K - k0);
    for (int k = 0; k < kn; ++k) {
      cd e = cis2pi(frac_mul(di, sth[k]));
      acc.x = fma(sga[k], e.x, acc.x);
      acc.y = fma(sga[k], e.y, acc.y);
    }
  }
  if (i < in.N) {
    if (i == 0) { acc.x += beta[b]; acc.y = 0.0; }
    c[in.off + i] = acc;
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
                                  cd* c, int B, int maxN, hipStream_t st) {
  dim3 grid((maxN + 255) / 256, B);
  hipLaunchKernelGGL(k_toeplitz_column, grid, dim3(256), 0, st, info, req, Kcnt, theta, gamma,
                     beta, c);
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
