// a4: w = C^{-1} y through the Gohberg-Semencul factors as FFT convolutions;
// a5: diagonal sums omega as FFT correlations of rho with its moments.
// One workgroup per instance; the FFT array of P points lives in LDS.
#include "sfls_kernels.hpp"
#include "k_launch.hpp"

namespace sfls {

constexpr int CONV_NT = 512;

struct cd3x2 { cd3 p, q; };
struct cd4x2 { cd4 p, q; };

// W_P^m = exp(-j 2 pi m / P) evaluated from the exact fraction (m mod P) / P:
// the points of a pointwise step need it at scattered m, where a table would
// be gathered one cache line per lane
__device__ __forceinline__ cd w_pow(int64_t m, int logP) {
  const int64_t P = (int64_t)1 << logP;
  return cconj(cis_frac(m & (P - 1), P));
}

// W_P^m = exp(-j 2 pi m / P) from the table tw[k] = exp(-j 2 pi k / 2^logtw), k < 2^(logtw-1)
__device__ __forceinline__ cd tw_pow(const cd* __restrict__ tw, int logtw, int64_t m, int logP) {
  const int64_t P = (int64_t)1 << logP;
  m &= (P - 1);
  const int64_t half = P >> 1;
  if (m >= half) {
    cd w = tw[(m - half) << (logtw - logP)];
    return cd{-w.x, -w.y};
  }
  return tw[m << (logtw - logP)];
}

template <typename YT> __device__ __forceinline__ cd load_y(const YT* y, int64_t i);
template <> __device__ __forceinline__ cd load_y<cd>(const cd* y, int64_t i) { return y[i]; }
template <> __device__ __forceinline__ cd load_y<cf>(const cf* y, int64_t i) { return to_d(y[i]); }

// ---------------------------------------------------------------------------
// a4.  With rho~_m = rho_{N-1-m} and y^_k = y_{N-1-k} (reversals):
//   u1 = T1 y      : u1_i = (rho~ * y^)_{N-1-i}
//   v1 = T0^H y    : v1_i = (conj(rho) * y^)_{N-2-i}   (v1_{N-1} = 0)
//   u2 = T1^H u1   = (conj(rho~) * u1)_i
//   v2 = T0 v1     = (rho * v1)_{i-1}
//   w  = (u2 - v2) / delta_{N-1}                       (eq. gohberg-semencul)
// All convolutions are length-P circular ones (P >= 2N-1, no wrap into the
// kept indices), transformed in LDS (padded layout).  Spectra are kept in
// bit-reversed order (DIF forward, DIT inverse), and the spectra of the reversed / conjugated rho are read off
// A = FFT(rho) at the negated frequency:
//   FFT(rho~)(f) = W^{f(N-1)} A(-f),  FFT(conj rho)(f) = conj A(-f),
//   FFT(conj rho~)(f) = W^{f(N-1)} conj A(f),  delay by one: W^f.
// Scratch per instance (4 P points): A, Y/U, X1, X2.  A stays for a5.
// ---------------------------------------------------------------------------
template <typename YT>
__global__ __launch_bounds__(CONV_NT) void k_gs_apply(const InstInfo* __restrict__ info,
                                                      const int32_t* __restrict__ req,
                                                      const YT* __restrict__ y,
                                                      const cd* __restrict__ rho,
                                                      const double* __restrict__ delta,
                                                      const cd* __restrict__ tw, int logtw,
                                                      const cd* __restrict__ tws,
                                                      cd* __restrict__ scratch, cd* __restrict__ w,
                                                      double* __restrict__ yCy,
                                                      double* __restrict__ ww,
                                                      const int32_t* __restrict__ order,
                                                      Vecs vv) {
  const int bi = order ? order[blockIdx.x] : blockIdx.x;
  if (req && !(req[bi] & REQ_EVAL)) return;
  const InstInfo in = info[bi];
  const int N = in.N, P = in.P, logP = in.logP;
  extern __shared__ cd lds_sh[];
  __shared__ double red[2 * (CONV_NT / 64)];
  __shared__ cd s_tw[FFT_TWL];
  const int tid = threadIdx.x;
  load_tw_head<CONV_NT>(s_tw, tws);
  const cd* rb = rho + in.off;
  cd* A = scratch + in.poff;
  cd* Y = A + P;
  cd* X1 = Y + P;
  cd* X2 = X1 + P;
  const double invP = 1.0 / (double)P;

  // The transform buffer: LDS, or for P > CONV_LDS_P the instance's scratch
  // after its four P blocks (the same passes, on global memory).
  auto body = [&](cd* __restrict__ lds) __attribute__((always_inline)) {
    // The h = 1 stage of each transform (the last of a forward one, the first
    // of an inverse one) runs on bit-reversed pairs (2g, 2g+1) inside the
    // neighbouring loop instead of an LDS pass of its own.  Its only twiddle
    // is W_2^0 = 1, so the butterfly is a plain sum and difference (no table
    // read: the LDS twiddle table is not yet published to every wave when
    // this lambda is entered).  A pair belongs to one thread; other threads'
    // indices are touched only after a barrier.
    auto dif_pair = [&](int g, cd& a, cd& b) {
      const cd u = lds[pidx(2 * g)], v = lds[pidx(2 * g + 1)];
      a = cadd(u, v);
      b = csub(u, v);
    };
    auto dit_pair = [&](int g, cd a, cd b) {
      lds[pidx(2 * g)] = cadd(a, b);
      lds[pidx(2 * g + 1)] = csub(a, b);
    };
    auto spectrum_to = [&](cd* __restrict__ dst) {
      for (int g = tid; g < P / 2; g += CONV_NT) {
        cd a, b;
        dif_pair(g, a, b);
        dst[2 * g] = a;
        dst[2 * g + 1] = b;
      }
      __syncthreads();
    };
    // (1) A = FFT(rho), shared by the vectors
    auto to_lds = [&](int t, cd v) { lds[pidx(t)] = v; };
    batched_for<8>(tid, CONV_NT, P, [&](int t) { return (t < N) ? rb[t] : cd{0.0, 0.0}; }, to_lds);
    __syncthreads();
    dif_fftn<CONV_NT>(lds, lds, 1, logP, false, false, s_tw, tws, 1);
    spectrum_to(A);
    // y^H C^{-1} y and ||w||^2 summed over the vectors
    double acc[2] = {0.0, 0.0};
    for (int gv = 0; gv < vv.G; ++gv) {
    const YT* yb = y + gv * vv.ystride + in.off;
    cd* wout = w + gv * vv.wstride + in.off;
    if (gv > 0) __syncthreads();  // the last vector's w read the transform buffer
    // (2) Y = FFT(y^)
    batched_for<8>(tid, CONV_NT, P,
                   [&](int t) { return (t < N) ? load_y(yb, N - 1 - t) : cd{0.0, 0.0}; }, to_lds);
    __syncthreads();
    dif_fftn<CONV_NT>(lds, lds, 1, logP, false, false, s_tw, tws, 1);
    spectrum_to(Y);
    // (3) u1 from FFT(rho~) . Y
    batched_for<2>(tid, CONV_NT, P / 2, [&](int g) {
      cd3 r[2];
      for (int k = 0; k < 2; ++k) {
        const int p = 2 * g + k;
        const int f = bitrev(p, logP);
        const int pm = bitrev((P - f) & (P - 1), logP);
        r[k] = cd3{w_pow((int64_t)f * (N - 1), logP), A[pm], Y[p]};
      }
      return cd3x2{r[0], r[1]};
    }, [&](int g, cd3x2 v) {
      dit_pair(g, cmul(cmul(v.p.a, v.p.b), v.p.c), cmul(cmul(v.q.a, v.q.b), v.q.c));
    });
    __syncthreads();
    dit_fftn<CONV_NT>(lds, lds, 1, logP, true, true, s_tw, tws, 1);
    for (int i = tid; i < N; i += CONV_NT) X1[i] = cscale(lds[pidx(N - 1 - i)], invP);
    __syncthreads();
    // (4) v1 from conj(A(-f)) . Y
    batched_for<2>(tid, CONV_NT, P / 2, [&](int g) {
      cd2 r[2];
      for (int k = 0; k < 2; ++k) {
        const int p = 2 * g + k;
        const int f = bitrev(p, logP);
        const int pm = bitrev((P - f) & (P - 1), logP);
        r[k] = cd2{A[pm], Y[p]};
      }
      return cd4{r[0].a, r[0].b, r[1].a, r[1].b};
    }, [&](int g, cd4 v) { dit_pair(g, cmul(cconj(v.a), v.b), cmul(cconj(v.c), v.d)); });
    __syncthreads();
    dit_fftn<CONV_NT>(lds, lds, 1, logP, true, true, s_tw, tws, 1);
    for (int i = tid; i < N; i += CONV_NT)
      X2[i] = (i <= N - 2) ? cscale(lds[pidx(N - 2 - i)], invP) : cd{0.0, 0.0};
    __syncthreads();
    // (5) U = FFT(u1) -> Y
    batched_for<8>(tid, CONV_NT, P, [&](int t) { return (t < N) ? X1[t] : cd{0.0, 0.0}; }, to_lds);
    __syncthreads();
    dif_fftn<CONV_NT>(lds, lds, 1, logP, false, false, s_tw, tws, 1);
    spectrum_to(Y);
    // (6) V = FFT(v1), kept in LDS (its h = 1 stage in step 7)
    batched_for<8>(tid, CONV_NT, P, [&](int t) { return (t < N) ? X2[t] : cd{0.0, 0.0}; }, to_lds);
    __syncthreads();
    dif_fftn<CONV_NT>(lds, lds, 1, logP, false, false, s_tw, tws, 1);
    // (7) W = FFT(conj rho~) U - W^f A V
    batched_for<2>(tid, CONV_NT, P / 2, [&](int g) {
      cd4 r[2];
      for (int k = 0; k < 2; ++k) {
        const int p = 2 * g + k;
        const int f = bitrev(p, logP);
        r[k] = cd4{A[p], Y[p], w_pow((int64_t)f * (N - 1), logP), w_pow(f, logP)};
      }
      return cd4x2{r[0], r[1]};
    }, [&](int g, cd4x2 v) {
      cd V0, V1;
      dif_pair(g, V0, V1);
      const cd t10 = cmul(cmul(v.p.c, cconj(v.p.a)), v.p.b);
      const cd t20 = cmul(cmul(v.p.d, v.p.a), V0);
      const cd t11 = cmul(cmul(v.q.c, cconj(v.q.a)), v.q.b);
      const cd t21 = cmul(cmul(v.q.d, v.q.a), V1);
      dit_pair(g, csub(t10, t20), csub(t11, t21));
    });
    __syncthreads();
    dit_fftn<CONV_NT>(lds, lds, 1, logP, true, true, s_tw, tws, 1);
    const double sc = invP / delta[in.off + N - 1];
    batched_for<8>(tid, CONV_NT, N, [&](int i) { return load_y(yb, i); }, [&](int i, cd yi) {
      const cd wi = cscale(lds[pidx(i)], sc);
      wout[i] = wi;
      acc[0] += fma(yi.x, wi.x, yi.y * wi.y);  // Re(conj(y) w)
      acc[1] += cabs2(wi);
    });
    }
    block_sum<CONV_NT, 2>(acc, red);
    if (tid == 0) {
      if (yCy) yCy[bi] = acc[0];
      if (ww) ww[bi] = acc[1];
    }
  };
  if (P > CONV_LDS_P) body(scratch + in.poff + 4 * (int64_t)P);
  else body(lds_sh);
}

// ---------------------------------------------------------------------------
// a5.  Diagonal sums as correlations.  With G_a the spectra of
// f_a(q) = (q - c)^a rho_q (c = (N-1)/2; f_0 spectrum = A from a4) and a
// polynomial weight W(q, p) = sum_ab C[a][b] (q-c)^a (p-c)^b derived from the
// Gohberg-Semencul structure (Appendix B):
//   omega(i) = delta^{-1} sum_q W(q, q+i) rho_q conj(rho_{q+i})
//            = delta^{-1} conj( IFFT( sum_ab C[a][b] G_b conj(G_a) ) (i) ).
// `which` selects the outputs (bit0 s, bit1 t, bit2 v, bit3 x).  omega_s is
// always written to oms (P points, lag i at i mod P) for the grid stage; the
// API outputs (2N-1 points, lag i at i+N-1) are written when non-NULL.
// Scratch: G_0 = A (from a4 when have_g0, else computed here) and the three
// following P-blocks for G_1..G_3.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(CONV_NT) void k_omega(const InstInfo* __restrict__ info,
                                                   const int32_t* __restrict__ req,
                                                   const cd* __restrict__ rho,
                                                   const double* __restrict__ delta,
                                                   const SepCoef* __restrict__ coef,
                                                   const cd* __restrict__ tws,
                                                   cd* __restrict__ scratch, int which,
                                                   int have_g0,
                                                   cd* __restrict__ oms, cd* __restrict__ o_s,
                                                   cd* __restrict__ o_t, cd* __restrict__ o_v,
                                                   cd* __restrict__ o_x,
                                                   const int32_t* __restrict__ order) {
  const int bi = order ? order[blockIdx.x] : blockIdx.x;
  if (req && !(req[bi] & REQ_GRID)) return;
  const InstInfo in = info[bi];
  const int N = in.N, P = in.P, logP = in.logP;
  extern __shared__ cd lds_sh[];
  __shared__ cd s_tw[FFT_TWL];
  const int tid = threadIdx.x;
  load_tw_head<CONV_NT>(s_tw, tws);
  const cd* rb = rho + in.off;
  cd* G0 = scratch + in.poff;  // G_a at G0 + a P
  const int amax = (which & ~1) ? 3 : 1;
  const double cN = 0.5 * (double)(N - 1);
  // The transform buffer: LDS, or for P > CONV_LDS_P the instance's scratch
  // after its four P blocks (the same passes, on global memory).
  auto body = [&](cd* __restrict__ lds) __attribute__((always_inline)) {
    for (int a = have_g0 ? 1 : 0; a <= amax; ++a) {
      batched_for<8>(tid, CONV_NT, P, [&](int t) { return (t < N) ? rb[t] : cd{0.0, 0.0}; },
                     [&](int t, cd v) {
        const double x = (double)t - cN;
        double m = 1.0;
        for (int e = 0; e < a; ++e) m *= x;
        lds[pidx(t)] = cscale(v, m);
      });
      __syncthreads();
      dif_fftn<CONV_NT>(lds, lds, 1, logP, false, false, s_tw, tws);
      for (int t = tid; t < P; t += CONV_NT) G0[(int64_t)a * P + t] = lds[pidx(t)];
      __syncthreads();
    }
    const SepCoef* cfp = coef + bi;
    const double scale = 1.0 / ((double)P * delta[in.off + N - 1]);
    for (int qk = 0; qk < 4; ++qk) {
      if (!(which & (1 << qk))) continue;
      const double* C = cfp->c[qk];
      const int am = (qk == 0) ? 1 : 3;
      cd* outq = qk == 0 ? o_s : (qk == 1 ? o_t : (qk == 2 ? o_v : o_x));
      batched_for<2>(tid, CONV_NT, P, [&](int p) {
        cd4 g;
        g.a = G0[p];
        g.b = (am >= 1) ? G0[(int64_t)P + p] : cd{0.0, 0.0};
        g.c = (am >= 2) ? G0[(int64_t)2 * P + p] : cd{0.0, 0.0};
        g.d = (am >= 3) ? G0[(int64_t)3 * P + p] : cd{0.0, 0.0};
        return g;
      }, [&](int p, cd4 gg) {
        const cd g[4] = {gg.a, gg.b, gg.c, gg.d};
        cd acc{0.0, 0.0};
  #pragma unroll
        for (int a = 0; a < 4; ++a)
  #pragma unroll
          for (int b2 = 0; b2 < 4; ++b2) {
            const double cab = (a <= am && b2 <= am) ? C[a * 4 + b2] : 0.0;
            if (cab != 0.0) {
              const cd pr = cmulc(g[b2], g[a]);  // G_b conj(G_a)
              acc.x = fma(cab, pr.x, acc.x);
              acc.y = fma(cab, pr.y, acc.y);
            }
          }
        lds[pidx(p)] = acc;
      });
      __syncthreads();
      dit_fftn<CONV_NT>(lds, lds, 1, logP, true, true, s_tw, tws);
      for (int t = tid; t < P; t += CONV_NT) {
        // lag i = t for t < N, i = t - P for t > P - N
        const bool pos = t < N, neg = t > P - N;
        if (!pos && !neg) continue;
        const cd om = cscale(cconj(lds[pidx(t)]), scale);
        if (qk == 0 && oms) oms[in.poff + t] = om;
        if (outq) {
          const int i = pos ? t : t - P;
          outq[in.ooff + i + N - 1] = om;
        }
      }
      if (qk == 0 && oms) {
        for (int t = tid; t < P; t += CONV_NT)
          if (!(t < N) && !(t > P - N)) oms[in.poff + t] = cd{0.0, 0.0};
      }
      __syncthreads();
    }
  };
  if (P > CONV_LDS_P) body(scratch + in.poff + 4 * (int64_t)P);
  else body(lds_sh);
}

// ---------------------------------------------------------------------------
// a3 refinement.  The superfast recursion's generator is refined by one step
// of iterative refinement on the last column of C^{-1}: with x0 = rho /
// delta_{N-1},
//   r = e_{N-1} - C x0            (k_gen_residual: length-P circular
//                                  convolution with the Hermitian extension
//                                  h_t = c_t, h_{P-t} = conj(c_t) of c)
//   dx = C~^{-1} r                (k_gs_apply with the unrefined generator)
//   x1 = x0 + dx,  rho <- x1 / x1_{N-1},  delta_{N-1} <- 1 / x1_{N-1}
//                                 (k_gen_update; x1_{N-1} is real).
// Instances whose factorisation failed are left alone.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(CONV_NT) void k_gen_residual(const InstInfo* __restrict__ info,
                                                          const int32_t* __restrict__ req,
                                                          const int32_t* __restrict__ status,
                                                          const cd* __restrict__ c,
                                                          const cd* __restrict__ rho,
                                                          const double* __restrict__ delta,
                                                          const cd* __restrict__ tws,
                                                          cd* __restrict__ scratch,
                                                          cd* __restrict__ r,
                                                          const int32_t* __restrict__ order) {
  const int bi = order ? order[blockIdx.x] : blockIdx.x;
  if (req && !(req[bi] & REQ_EVAL)) return;
  if (status && status[bi] != 0) return;
  const InstInfo in = info[bi];
  const int N = in.N, P = in.P, logP = in.logP;
  extern __shared__ cd lds_sh[];
  __shared__ cd s_tw[FFT_TWL];
  const int tid = threadIdx.x;
  load_tw_head<CONV_NT>(s_tw, tws);
  const cd* cb = c + in.off;
  const cd* rb = rho + in.off;
  cd* H = scratch + in.poff;
  const double inv_d = 1.0 / delta[in.off + N - 1];
  // The transform buffer: LDS, or for P > CONV_LDS_P the instance's scratch
  // after its four P blocks (the same passes, on global memory).
  auto body = [&](cd* __restrict__ lds) __attribute__((always_inline)) {
    batched_for<8>(tid, CONV_NT, P, [&](int t) {
      cd v{0.0, 0.0};
      if (t < N) v = cb[t];
      else if (t > P - N) v = cconj(cb[P - t]);
      return v;
    }, [&](int t, cd v) { lds[pidx(t)] = v; });
    __syncthreads();
    dif_fftn<CONV_NT>(lds, lds, 1, logP, false, false, s_tw, tws);
    for (int t = tid; t < P; t += CONV_NT) H[t] = lds[pidx(t)];
    __syncthreads();
    batched_for<8>(tid, CONV_NT, P, [&](int t) { return (t < N) ? cscale(rb[t], inv_d) : cd{0.0, 0.0}; },
                   [&](int t, cd v) { lds[pidx(t)] = v; });
    __syncthreads();
    dif_fftn<CONV_NT>(lds, lds, 1, logP, false, false, s_tw, tws);
    batched_for<8>(tid, CONV_NT, P, [&](int p) { return H[p]; },
                   [&](int p, cd h) { lds[pidx(p)] = cmul(lds[pidx(p)], h); });
    __syncthreads();
    dit_fftn<CONV_NT>(lds, lds, 1, logP, true, true, s_tw, tws);
    const double invP = 1.0 / (double)P;
    for (int i = tid; i < N; i += CONV_NT) {
      const cd cx = cscale(lds[pidx(i)], invP);
      r[in.off + i] = cd{(i == N - 1 ? 1.0 : 0.0) - cx.x, -cx.y};
    }
  };
  if (P > CONV_LDS_P) body(scratch + in.poff + 4 * (int64_t)P);
  else body(lds_sh);
}

__global__ __launch_bounds__(CONV_NT) void k_gen_update(const InstInfo* __restrict__ info,
                                                        const int32_t* __restrict__ req,
                                                        const int32_t* __restrict__ status,
                                                        cd* __restrict__ rho,
                                                        double* __restrict__ delta,
                                                        const cd* __restrict__ dx,
                                                        const int32_t* __restrict__ order) {
  const int bi = order ? order[blockIdx.x] : blockIdx.x;
  if (req && !(req[bi] & REQ_EVAL)) return;
  if (status && status[bi] != 0) return;
  const InstInfo in = info[bi];
  const int N = in.N;
  cd* rb = rho + in.off;
  const cd* db = dx + in.off;
  __shared__ double s_inv_d, s_scale;
  if (threadIdx.x == 0) {
    const double inv_d = 1.0 / delta[in.off + N - 1];
    const double xl = fma(rb[N - 1].x, inv_d, db[N - 1].x);  // x1_{N-1}, real
    s_inv_d = inv_d;
    s_scale = 1.0 / xl;
  }
  __syncthreads();
  const double inv_d = s_inv_d, sc = s_scale;
  for (int i = threadIdx.x; i < N - 1; i += CONV_NT) {
    const cd x1{fma(rb[i].x, inv_d, db[i].x), fma(rb[i].y, inv_d, db[i].y)};
    rb[i] = cscale(x1, sc);
  }
  if (threadIdx.x == 0) {
    rb[N - 1] = cd{1.0, 0.0};
    delta[in.off + N - 1] = sc;
  }
}

hipError_t launch_gen_refine(const InstInfo* info, const int32_t* req, const int32_t* status,
                             const cd* c, cd* rho, double* delta, const cd* tw, int logtw,
                             const cd* tws, cd* scratch, cd* r, cd* dx, int B, int maxP,
                             hipStream_t st, const int32_t* order) {
  const size_t shm = (size_t)padded(maxP < CONV_LDS_P ? maxP : CONV_LDS_P) * sizeof(cd);
  (void)hipFuncSetAttribute((const void*)k_gen_residual,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  hipLaunchKernelGGL(k_gen_residual, dim3(B), dim3(CONV_NT), shm, st, info, req, status, c, rho,
                     delta, tws, scratch, r, order);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_gs_apply(info, req, r, 1, rho, delta, tw, logtw, tws, scratch, dx, nullptr, nullptr,
                      B, maxP, st, order);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gen_update, dim3(B), dim3(CONV_NT), 0, st, info, req, status, rho, delta,
                     dx, order);
  return hipGetLastError();
}

hipError_t launch_gs_apply(const InstInfo* info, const int32_t* req, const void* y, int ydtype,
                           const cd* rho, const double* delta, const cd* tw, int logtw,
                           const cd* tws, cd* scratch, cd* w, double* yCy, double* ww, int B, int maxP,
                           hipStream_t st, const int32_t* order, Vecs vv) {
  const size_t shm = (size_t)padded(maxP < CONV_LDS_P ? maxP : CONV_LDS_P) * sizeof(cd);
  if (ydtype == 1) {
    (void)hipFuncSetAttribute((const void*)k_gs_apply<cd>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)shm);
    hipLaunchKernelGGL(k_gs_apply<cd>, dim3(B), dim3(CONV_NT), shm, st, info, req, (const cd*)y,
                       rho, delta, tw, logtw, tws, scratch, w, yCy, ww, order, vv);
  } else {
    (void)hipFuncSetAttribute((const void*)k_gs_apply<cf>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)shm);
    hipLaunchKernelGGL(k_gs_apply<cf>, dim3(B), dim3(CONV_NT), shm, st, info, req, (const cf*)y,
                       rho, delta, tw, logtw, tws, scratch, w, yCy, ww, order, vv);
  }
  return hipGetLastError();
}

hipError_t launch_omega(const InstInfo* info, const int32_t* req, const cd* rho,
                        const double* delta, const SepCoef* coef, const cd* tws,
                        cd* scratch, int which, int have_g0, cd* oms, cd* o_s, cd* o_t,
                        cd* o_v, cd* o_x, int B, int maxP, hipStream_t st,
                        const int32_t* order) {
  const size_t shm = (size_t)padded(maxP < CONV_LDS_P ? maxP : CONV_LDS_P) * sizeof(cd);
  (void)hipFuncSetAttribute((const void*)k_omega, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  hipLaunchKernelGGL(k_omega, dim3(B), dim3(CONV_NT), shm, st, info, req, rho, delta, coef, tws,
                     scratch, which, have_g0, oms, o_s, o_t, o_v, o_x, order);
  return hipGetLastError();
}

}  // namespace sfls
