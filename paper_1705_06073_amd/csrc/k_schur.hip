// a3: the Gohberg-Semencul generator by a superfast (doubling) Schur
// recursion, O(N log^2 N) per instance (Sec. III cites the generalized Schur
// algorithm for this step).
//
// Generator of the Schur recursion at order n (residuals of the predictors):
//   U^(n)(i) = sum_j c_{i-j} a^(n)_j,   V^(n)(i) = sum_j c_{i-j} b^(n)_j,
// with U^(0)(i) = V^(0)(i) = c_i, V^(n)(n) = delta_n.  One step:
//   k = -U(n+1) / V(n),  [U; V](z) <- theta_k(z) [U; V](z),
//   theta_k(z) = [[1, k z], [conj(k), z]],
// and the predictors obey the same map, so after N-1 steps
//   [a; b](z) = Theta(z) [1; 1],  rho = b = Theta_21 + Theta_22.
// Theta over m steps is stored as four polynomials of m coefficients,
//   P11 = Theta_11, P12 = Theta_12 / z, P21 = Theta_21, P22 = Theta_22 / z,
// all of degree <= m-1, so every product below fits an FFT of size >= m
// without wrap-around.
//
// Recursion S(n0, m) on the window u[r] = U^(n0)(n0+1+r), v[r] = V^(n0)(n0+r),
// r < m:
//   leaf (m <= 64): one wave runs the m steps (lane r holds u[r], v[r] and the
//     r-th coefficient of the four polynomials);
//   otherwise m1 = m/2: S(n0, m1) on the window prefix -> Theta1;
//     MID:  the right half's window from Theta1 applied to (u, v):
//           P1 = P11 * u + P12 * v,  P2 = P21 * u + P22 * v  (convolutions),
//           u2[r] = P1[m1 + r], v2[r] = P2[m1 - 1 + r];
//     S(n0+m1, m-m1) on (u2, v2) -> Theta2;
//     POST: Theta = Theta2 Theta1 (shifted form, z = e^{-j2pi f/F} per bin).
// The host flattens the recursion of each N into an action list; one
// workgroup per instance walks it.  Spectra stay in bit-reversed order.
#include "k_launch.hpp"
#include "sfls_kernels.hpp"

namespace sfls {

constexpr int SCH_NT = 256;
constexpr int SCH_LEAF = 64;

__device__ __forceinline__ double shr1d(double v) {
  int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xF, 0xF, false);
  int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ cd shr1c(cd v) { return cd{shr1d(v.x), shr1d(v.y)}; }
__device__ __forceinline__ cd readlane_c(cd v, int l) { return cd{readlane_f64(v.x, l), readlane_f64(v.y, l)}; }

// two radix-2 FFTs over the same stages (shared barriers)
template <int NT>
__device__ void dif_fft2(cd* x, cd* y, int logn, int sgn, const cd* __restrict__ tws) {
  const int n = 1 << logn;
  for (int lh = logn - 1; lh >= 0; --lh) {
    const int h = 1 << lh;
    for (int b = threadIdx.x; b < n; b += NT) {
      cd* z = (b < (n >> 1)) ? x : y;
      const int bb = b & ((n >> 1) - 1);
      const int pos = bb & (h - 1);
      const int i = ((bb >> lh) << (lh + 1)) + pos;
      const int j = i + h;
      cd u = z[i], v = z[j];
      cd w = tws[h + pos];
      if (sgn > 0) w.y = -w.y;
      z[i] = cadd(u, v);
      z[j] = cmul(csub(u, v), w);
    }
    __syncthreads();
  }
}

template <int NT>
__device__ void dit_fft2(cd* x, cd* y, int logn, int sgn, const cd* __restrict__ tws) {
  const int n = 1 << logn;
  for (int lh = 0; lh < logn; ++lh) {
    const int h = 1 << lh;
    for (int b = threadIdx.x; b < n; b += NT) {
      cd* z = (b < (n >> 1)) ? x : y;
      const int bb = b & ((n >> 1) - 1);
      const int pos = bb & (h - 1);
      const int i = ((bb >> lh) << (lh + 1)) + pos;
      const int j = i + h;
      cd w = tws[h + pos];
      if (sgn > 0) w.y = -w.y;
      cd u = z[i], v = cmul(z[j], w);
      z[i] = cadd(u, v);
      z[j] = csub(u, v);
    }
    __syncthreads();
  }
}

// W_F^f = exp(-j 2 pi f / F) for the bin at bit-reversed position p
__device__ __forceinline__ cd zbin(const cd* __restrict__ tw, int logtw, int p, int logF) {
  const int f = bitrev(p, logF);
  const int F = 1 << logF;
  if (f >= (F >> 1)) {
    const cd w = tw[(f - (F >> 1)) << (logtw - logF)];
    return cd{-w.x, -w.y};
  }
  return tw[f << (logtw - logF)];
}

__global__ __launch_bounds__(SCH_NT) void k_schur(const InstInfo* __restrict__ info,
                                                  const int32_t* __restrict__ req,
                                                  const SchurLayout* __restrict__ lay,
                                                  const SchurAct* __restrict__ acts,
                                                  const cd* __restrict__ c,
                                                  const cd* __restrict__ tw, int logtw,
                                                  const cd* __restrict__ tws,
                                                  cd* __restrict__ scratch, cd* __restrict__ rho,
                                                  double* __restrict__ delta_out,
                                                  double* __restrict__ logdet,
                                                  int32_t* __restrict__ status,
                                                  int64_t* __restrict__ failed) {
  const int bi = blockIdx.x;
  if (req && !(req[bi] & REQ_EVAL)) return;
  const InstInfo in = info[bi];
  const SchurLayout& L = lay[bi];  // read through uniform addresses (scalar loads)
  const int N = in.N;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  extern __shared__ cd lds[];
  cd* A = lds;
  cd* Bf = lds + L.Fmax;
  __shared__ double s_logdet;
  __shared__ int s_fail;
  const cd* cb = c + in.off;
  cd* scr = scratch + L.scr_off;
  double* dl = delta_out ? delta_out + in.off : nullptr;
  if (tid == 0) {
    s_logdet = log(cb[0].x);
    s_fail = (cb[0].x > 0.0 && isfinite(cb[0].x)) ? -1 : 0;
    if (dl) dl[0] = cb[0].x;
  }
  __syncthreads();
  if (N == 1 || s_fail >= 0) {
    if (tid == 0) {
      rho[in.off] = cd{1.0, 0.0};
      if (logdet) logdet[bi] = (s_fail < 0) ? s_logdet : __builtin_nan("");
      if (status) status[bi] = (s_fail < 0) ? 0 : -4;
      if (failed) failed[bi] = s_fail;
    }
    return;
  }
  const int nact = __builtin_amdgcn_readfirstlane(L.nact);
  const SchurAct* my_acts = acts + L.act_off;
  for (int ai = 0; ai < nact; ++ai) {
    SchurAct act;
    act.type = __builtin_amdgcn_readfirstlane(my_acts[ai].type);
    act.n0 = __builtin_amdgcn_readfirstlane(my_acts[ai].n0);
    act.m = __builtin_amdgcn_readfirstlane(my_acts[ai].m);
    act.m1 = __builtin_amdgcn_readfirstlane(my_acts[ai].m1);
    act.level = __builtin_amdgcn_readfirstlane(my_acts[ai].level);
    act.side = __builtin_amdgcn_readfirstlane(my_acts[ai].side);
    act.win_level = __builtin_amdgcn_readfirstlane(my_acts[ai].win_level);
    act.logF = __builtin_amdgcn_readfirstlane(my_acts[ai].logF);
    const int m = act.m, m1 = act.m1, m2 = m - m1;
    // window of this node
    const cd* u;
    const cd* v;
    if (act.win_level < 0) { u = cb + 1; v = cb; }
    else { u = scr + L.win[act.win_level]; v = u + L.mmax[act.win_level]; }
    if (act.type == SCH_LEAF_ACT || act.type == SCH_ROOT_LEAF) {
      if (wv == 0) {
        cd U = (lane < m) ? u[lane] : cd{0.0, 0.0};
        cd V = (lane < m) ? v[lane] : cd{0.0, 0.0};
        double dlt = readlane_f64(V.x, 0);
        double inv = 1.0 / dlt;
        double my_dn = 1.0;   // delta_{n0+1+lane}, kept by lane s at step s
        int fail = -1;
        cd T11{0.0, 0.0}, T12{0.0, 0.0}, T21{0.0, 0.0}, T22{0.0, 0.0};
        for (int s = 0; s < m; ++s) {
          const cd Us = readlane_c(U, s);
          const cd k{-Us.x * inv, -Us.y * inv};
          const double q = 1.0 - cabs2(k);
          const double dn = dlt * q;
          // 1/delta_{n+1} = (1/delta_n) / q: hardware reciprocal + one Newton step
          const double r0 = __builtin_amdgcn_rcp(q);
          const double r1 = fma(r0, fma(-q, r0, 1.0), r0);
          const bool bad = !(dn > 0.0) || !isfinite(dn);
          if (bad && fail < 0) fail = act.n0 + s + 1;
          const cd Ush = shr1c(U), Vsh = shr1c(V);
          U = cfma(k, V, U);            // U(i) + k V(i-1): same lane
          V = cfmac(Ush, k, Vsh);       // V(i-1) + conj(k) U(i): both from lane r-1
          if (s == 0) {
            const bool l0 = lane == 0;
            T11 = cd{l0 ? 1.0 : 0.0, 0.0};
            T12 = l0 ? k : cd{0.0, 0.0};
            T21 = l0 ? cconj(k) : cd{0.0, 0.0};
            T22 = cd{l0 ? 1.0 : 0.0, 0.0};
          } else {
            const cd S21 = shr1c(T21), S22 = shr1c(T22);
            const cd o11 = T11, o12 = T12;
            T11 = cfma(k, S21, o11);      // P11 + k z P21
            T12 = cfma(k, S22, o12);      // P12 + k z P22
            T21 = cfmac(o11, k, S21);     // conj(k) P11 + z P21
            T22 = cfmac(o12, k, S22);     // conj(k) P12 + z P22
          }
          if (lane == s) my_dn = dn;
          dlt = dn;
          inv = inv * r1;
        }
        // pivots and their logs, one per lane
        double lg = 0.0;
        if (lane < m) {
          if (dl) dl[act.n0 + 1 + lane] = my_dn;
          lg = log(my_dn);
        }
        const double lsum = wave_sum(lg);
        if (lane == 0) {
          s_logdet += lsum;
          if (fail >= 0) s_fail = fail;
        }
        if (act.type == SCH_ROOT_LEAF) {
          // rho = P21 + z P22 (degree <= m = N-1 <= 63 < 64 lanes)
          const cd zP22 = shr1c(T22);
          if (lane < N) rho[in.off + lane] = cadd(T21, zP22);
        } else {
          cd* R = scr + L.res[act.level] + (int64_t)act.side * 4 * L.mmax[act.level];
          const int st = L.mmax[act.level];
          if (lane < m) {
            R[lane] = T11;
            R[st + lane] = T12;
            R[2 * st + lane] = T21;
            R[3 * st + lane] = T22;
          }
        }
      }
      __syncthreads();
      if (s_fail >= 0) break;
      continue;
    }
    const int logF = act.logF, F = 1 << logF;
    const double invF = 1.0 / (double)F;
    if (act.type == SCH_MID) {
      // spectra of Theta1 (left child, m1 coefficients per polynomial)
      const int cl = act.level + 1;
      const cd* T1 = scr + L.res[cl];
      const int st1 = L.mmax[cl];
      cd* S = scr + L.spec[act.level];
      for (int q = 0; q < 4; q += 2) {
        for (int t = tid; t < F; t += SCH_NT) {
          A[t] = (t < m1) ? T1[q * st1 + t] : cd{0.0, 0.0};
          Bf[t] = (t < m1) ? T1[(q + 1) * st1 + t] : cd{0.0, 0.0};
        }
        __syncthreads();
        dif_fft2<SCH_NT>(A, Bf, logF, -1, tws);
        for (int t = tid; t < F; t += SCH_NT) {
          S[(int64_t)q * F + t] = A[t];
          S[(int64_t)(q + 1) * F + t] = Bf[t];
        }
        __syncthreads();
      }
      // window spectra
      for (int t = tid; t < F; t += SCH_NT) {
        A[t] = (t < m) ? u[t] : cd{0.0, 0.0};
        Bf[t] = (t < m) ? v[t] : cd{0.0, 0.0};
      }
      __syncthreads();
      dif_fft2<SCH_NT>(A, Bf, logF, -1, tws);
      for (int p = tid; p < F; p += SCH_NT) {
        const cd fu = A[p], fv = Bf[p];
        const cd s11 = S[p], s12 = S[F + p], s21 = S[2 * F + p], s22 = S[3 * F + p];
        A[p] = cfma(s12, fv, cmul(s11, fu));
        Bf[p] = cfma(s22, fv, cmul(s21, fu));
      }
      __syncthreads();
      dit_fft2<SCH_NT>(A, Bf, logF, +1, tws);
      // right child's window
      cd* W2 = scr + L.win[cl];
      const int stw = L.mmax[cl];
      for (int r = tid; r < m2; r += SCH_NT) {
        W2[r] = cscale(A[m1 + r], invF);
        W2[stw + r] = cscale(Bf[m1 - 1 + r], invF);
      }
      __syncthreads();
      continue;
    }
    // POST / ROOT: Theta = Theta2 Theta1
    const int cl = act.level + 1;
    const cd* T2 = scr + L.res[cl] + (int64_t)4 * L.mmax[cl];  // right child's result
    const int st2 = L.mmax[cl];
    const cd* S = scr + L.spec[act.level];
    const bool root = act.type == SCH_ROOT;
    for (int row = root ? 1 : 0; row < 2; ++row) {
      for (int t = tid; t < F; t += SCH_NT) {
        A[t] = (t < m2) ? T2[(2 * row) * st2 + t] : cd{0.0, 0.0};
        Bf[t] = (t < m2) ? T2[(2 * row + 1) * st2 + t] : cd{0.0, 0.0};
      }
      __syncthreads();
      dif_fft2<SCH_NT>(A, Bf, logF, -1, tws);
      for (int p = tid; p < F; p += SCH_NT) {
        const cd a1 = A[p], a2 = cmul(Bf[p], zbin(tw, logtw, p, logF));  // z * second poly
        const cd s11 = S[p], s12 = S[F + p], s21 = S[2 * F + p], s22 = S[3 * F + p];
        const cd r1 = cfma(a2, s21, cmul(a1, s11));   // row . column 1
        const cd r2 = cfma(a2, s22, cmul(a1, s12));   // row . column 2 (shifted)
        if (root) {
          // rho = R21 + z R22'
          A[p] = cfma(r2, zbin(tw, logtw, p, logF), r1);
        } else {
          A[p] = r1;
          Bf[p] = r2;
        }
      }
      __syncthreads();
      if (root) {
        dit_fft<cd, SCH_NT>(A, logF, +1, tws);
        for (int t = tid; t < N; t += SCH_NT) rho[in.off + t] = cscale(A[t], invF);
        __syncthreads();
      } else {
        dit_fft2<SCH_NT>(A, Bf, logF, +1, tws);
        cd* R = scr + L.res[act.level] + (int64_t)act.side * 4 * L.mmax[act.level];
        const int st = L.mmax[act.level];
        for (int t = tid; t < m; t += SCH_NT) {
          R[(2 * row) * st + t] = cscale(A[t], invF);
          R[(2 * row + 1) * st + t] = cscale(Bf[t], invF);
        }
        __syncthreads();
      }
    }
  }
  if (tid == 0) {
    const bool ok = s_fail < 0;
    if (logdet) logdet[bi] = ok ? s_logdet : __builtin_nan("");
    if (status) status[bi] = ok ? 0 : -4;
    if (failed) failed[bi] = s_fail;
  }
}

hipError_t launch_schur(const InstInfo* info, const int32_t* req, const SchurLayout* lay,
                        const SchurAct* acts, const cd* c, const cd* tw, int logtw,
                        const cd* tws, cd* scratch,
                        cd* rho, double* delta, double* logdet, int32_t* status, int64_t* failed,
                        int B, int Fmax, hipStream_t st) {
  const size_t shm = 2 * (size_t)Fmax * sizeof(cd);
  (void)hipFuncSetAttribute((const void*)k_schur, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)shm);
  hipLaunchKernelGGL(k_schur, dim3(B), dim3(SCH_NT), shm, st, info, req, lay, acts, c, tw, logtw,
                     tws, scratch, rho, delta, logdet, status, failed);
  return hipGetLastError();
}

}  // namespace sfls
