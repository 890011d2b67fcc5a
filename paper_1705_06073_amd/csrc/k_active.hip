// a8: q, r, u, s, t, v, x at the active frequencies (and q, s at grid
// candidates for the FP64 re-check of activation decisions).
#include "sfls_kernels.hpp"
#include "k_launch.hpp"

namespace sfls {

constexpr int ACT_NT = 256;

// Exclusive prefix over instances of the number of work items:
// items(b) = (EVAL ? K[b] : 0) + (GRID ? ncand[b] : 0).  prefix has B+1 entries.
__global__ __launch_bounds__(1024) void k_item_scan(const int32_t* __restrict__ req,
                                                    const int32_t* __restrict__ Keval,
                                                    const int32_t* __restrict__ ncand, int B,
                                                    int32_t* __restrict__ prefix) {
  __shared__ int32_t part[1024];
  const int tid = threadIdx.x;
  const int per = (B + 1023) / 1024;
  const int b0 = tid * per;
  int32_t loc = 0;
  for (int b = b0; b < min(B, b0 + per); ++b) {
    const int32_t rq = req[b];
    loc += ((rq & REQ_EVAL) ? Keval[b] : 0) + ((rq & REQ_GRID) && ncand ? ncand[b] : 0);
  }
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
    const int32_t rq = req[b];
    run += ((rq & REQ_EVAL) ? Keval[b] : 0) + ((rq & REQ_GRID) && ncand ? ncand[b] : 0);
  }
  if (tid == 1023) prefix[B] = part[1023];
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
                                                   double* __restrict__ cs) {
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
    if (full) {
      for (int n = tid; n < N; n += ACT_NT) {
        const double dn = (double)n;
        const cd e = cconj(cis2pi(frac_mul(dn, th)));
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
      for (int n = tid; n < N; n += ACT_NT) {
        const double dn = (double)n;
        const cd e = cconj(cis2pi(frac_mul(dn, th)));
        const cd we = cmul(wb[n], e);
        const cd re = cmul(rb[n], e);
        const double x = dn - cN;
        acc[0] += we.x; acc[1] += we.y;
        acc[6] += re.x; acc[7] += re.y;
        acc[8] = fma(x, re.x, acc[8]); acc[9] = fma(x, re.y, acc[9]);
      }
    }
    block_sum<ACT_NT, 14>(acc, red);
    if (tid == 0) {
      const double idl = 1.0 / delta[in.off + N - 1];
      const SepCoef& cf = coef[bi];
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
    __syncthreads();
  }
}

hipError_t launch_active(const InstInfo* info, const int32_t* req, const int32_t* Keval,
                         const int32_t* ncand, int32_t* prefix, int B, const double* theta,
                         const int32_t* cand, const cd* w, const cd* rho, const double* delta,
                         const SepCoef* coef, cd* oq, cd* orr, cd* ou, cd* os, cd* ot, cd* ov,
                         cd* ox, cd* cq, double* cs, int nblocks, hipStream_t st) {
  hipLaunchKernelGGL(k_item_scan, dim3(1), dim3(1024), 0, st, req, Keval, ncand, B, prefix);
  hipLaunchKernelGGL(k_active, dim3(nblocks), dim3(ACT_NT), 0, st, info, req, Keval, prefix, B,
                     theta, cand, w, rho, delta, coef, oq, orr, ou, os, ot, ov, ox, cq, cs);
  return hipGetLastError();
}

}  // namespace sfls
