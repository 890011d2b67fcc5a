// ln|C| of an evaluation by the determinant lemma over the active set:
//   C = beta I + Psi Gamma Psi^H  =>
//   ln|C| = N ln beta + ln det(I_K + Gamma^{1/2} Psi^H Psi Gamma^{1/2} / beta),
// with the Gram matrix in closed form (Dirichlet kernel)
//   [Psi^H Psi]_{kl} = sum_{n<N} e^{j 2 pi n (theta_l - theta_k)}
//                    = e^{j pi (N-1) d} sin(pi N d) / sin(pi d),  d = theta_l - theta_k,
// and the K x K Hermitian positive-definite matrix (eigenvalues >= 1)
// factored as L D L^H in LDS.  This is the same quantity as sum_i ln delta_i
// of the factorisation (Sec. III-A); it is computed this way when K <= LEM_KMAX
// because it is accurate to a few ulp of N ln beta plus K eps cond(M), while
// the pivots of a long recursion carry O(N) accumulated rounding.  Larger
// active sets keep the factorisation's value.
#include "k_launch.hpp"
#include "sfls_kernels.hpp"

namespace sfls {

constexpr int LEM_NT = 256;
constexpr int LEM_KMAX = 96;

__global__ __launch_bounds__(LEM_NT) void k_logdet_lemma(const InstInfo* __restrict__ info,
                                                         const int32_t* __restrict__ req,
                                                         const int32_t* __restrict__ Kev,
                                                         const double* __restrict__ theta,
                                                         const double* __restrict__ gamma,
                                                         const double* __restrict__ beta,
                                                         const int32_t* __restrict__ status,
                                                         double* __restrict__ logdet,
                                                         const int32_t* __restrict__ order) {
  const int bi = order ? order[blockIdx.x] : blockIdx.x;
  if (!(req[bi] & REQ_EVAL)) return;
  if (status[bi] != 0) return;
  const int K = Kev[bi];
  if (K > LEM_KMAX) return;
  const InstInfo in = info[bi];  // components at in.koff
  const int N = in.N;
  const double be = beta[bi];
  const double* th = theta + in.koff;
  const double* ga = gamma + in.koff;
  constexpr int LD = LEM_KMAX + 1;  // padded row stride
  __shared__ cd M[LEM_KMAX * LD];
  __shared__ double s_sg[LEM_KMAX];
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  for (int k = tid; k < K; k += LEM_NT) s_sg[k] = sqrt(ga[k] / be);
  if (tid == 0) s_bad = 0;
  __syncthreads();
  // lower triangle (and diagonal) of M
  for (int e = tid; e < K * K; e += LEM_NT) {
    const int k = e / K, l = e % K;
    if (l > k) continue;
    double d = th[l] - th[k];
    d -= rint(d);  // (-1/2, 1/2]
    cd g;
    if (d == 0.0) {
      g = cd{(double)N, 0.0};
    } else {
      double sn, cs, sN, cN;
      sincospi(d, &sn, &cs);
      sincospi((double)N * d, &sN, &cN);
      double sph, cph;
      sincospi((double)(N - 1) * d, &sph, &cph);
      const double r = sN / sn;
      g = cd{cph * r, sph * r};
    }
    const double sc = s_sg[k] * s_sg[l];
    cd v = cscale(g, sc);
    if (k == l) v = cd{1.0 + v.x, 0.0};
    M[k * LD + l] = v;
  }
  __syncthreads();
  // right-looking LDL^H (no square roots): after step j, M_jj is the pivot d_j
  // and column j below it holds L_ij d_j; ln det M = sum_j ln d_j
  const int tr = tid >> 4, tc = tid & 15;  // 16 x 16 thread tile over (i, k)
  for (int j = 0; j < K - 1; ++j) {
    const double inv = 1.0 / M[j * LD + j].x;
    for (int i = j + 1 + tr; i < K; i += 16) {
      const cd mij = M[i * LD + j];
      for (int k = j + 1 + tc; k <= i; k += 16) {
        const cd mkj = M[k * LD + j];
        cd m = M[i * LD + k];
        // M_ik -= M_ij conj(M_kj) / d_j
        m.x -= (mij.x * mkj.x + mij.y * mkj.y) * inv;
        m.y -= (mij.y * mkj.x - mij.x * mkj.y) * inv;
        M[i * LD + k] = m;
      }
    }
    __syncthreads();
  }
  // ln d_j in parallel, then a block sum
  double acc[1] = {0.0};
  bool bad = false;
  for (int j = tid; j < K; j += LEM_NT) {
    const double dj = M[j * LD + j].x;
    bad |= !(dj > 0.0);
    acc[0] += log(dj);
  }
  if (bad) s_bad = 1;
  __shared__ double red[LEM_NT / 64];
  block_sum<LEM_NT, 1>(acc, red);
  if (tid == 0 && !s_bad) logdet[bi] = (double)N * log(be) + acc[0];
}

hipError_t launch_logdet_lemma(const InstInfo* info, const int32_t* req, const int32_t* Kev,
                               const double* theta, const double* gamma,
                               const double* beta, const int32_t* status, double* logdet, int B,
                               hipStream_t st, const int32_t* order) {
  hipLaunchKernelGGL(k_logdet_lemma, dim3(B), dim3(LEM_NT), 0, st, info, req, Kev, theta, gamma,
                     beta, status, logdet, order);
  return hipGetLastError();
}

}  // namespace sfls
