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
// Every section theta_k has the form [[A, B], [B#, A#]] with P#(z) the
// reversed conjugate z^deg conj(P(1/conj z)), and products keep that form, so
// in the shifted storage over m steps
//   P22[i] = conj(P11[m-1-i]),  P21[i] = conj(P12[m-1-i]),
// and for their spectra on F bins, S22(f) = W^(f(m-1)) conj(S11(f)) and
// S21(f) = W^(f(m-1)) conj(S12(f)) with W = exp(-j 2 pi / F).  POST therefore
// computes the first row of Theta2 Theta1 only and MID transforms P11 and P12
// only.
// The host flattens the recursion of each N into an action list; one
// workgroup per instance walks it.  Spectra stay in bit-reversed order.
#include "k_launch.hpp"
#include "sfls_kernels.hpp"

namespace sfls {

constexpr int SCH_NT = 256;
constexpr int SCH_LEAF = 64;
// transform merges of F <= 2^SCH_WAVE_LOG give each transform to one wave
constexpr int SCH_WAVE_LOG = 10;

// lane r <- lane r-1 (lane 0 <- 0)
__device__ __forceinline__ double shr1d(double v) {
  int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xF, 0xF, true);
  int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ cd shr1c(cd v) { return cd{shr1d(v.x), shr1d(v.y)}; }
// lane r <- lane r+1 (lane 63 <- 0)
__device__ __forceinline__ double shl1d(double v) {
  int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xF, 0xF, true);
  int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ cd shl1c(cd v) { return cd{shl1d(v.x), shl1d(v.y)}; }
__device__ __forceinline__ cd readlane_c(cd v, int l) { return cd{readlane_f64(v.x, l), readlane_f64(v.y, l)}; }

// Sliding-window block of RB outputs t0..t0+RB-1 of two convolutions,
//   acc[i] += sum_{j < J} a[j] x[t0+i-j] + b[j] y[t0+i-j],
// over LDS operands; x and y must be readable (zero where outside the
// polynomials) on [t0 - J - RB + 1, t0 + RB).  They are given as a row base
// and the padded index of the origin; element i of a padded row is stored at
// skew(i) = i + i / RB, so that lanes at output stride RB read distinct banks.
template <int RB>
__device__ __forceinline__ int skew(int i) {
  return RB > 1 ? i + (i >> (RB == 2 ? 1 : 2)) : i;
}
template <int RB>
__device__ __forceinline__ void conv2_block(const cd* a, const cd* xr, int xo, const cd* b,
                                            const cd* yr, int yo, int J, int t0,
                                            cd (&acc)[RB]) {
  constexpr int W = 2 * RB - 1;
  cd xv[W], yv[W];  // xv[k] = x[t0 - j0 + k - (RB - 1)]
#pragma unroll
  for (int k = 0; k < W; ++k) {
    xv[k] = xr[skew<RB>(xo + t0 + k - (RB - 1))];
    yv[k] = yr[skew<RB>(yo + t0 + k - (RB - 1))];
  }
  for (int j0 = 0; j0 < J; j0 += RB) {
#pragma unroll
    for (int jj = 0; jj < RB; ++jj) {
      if (j0 + jj < J) {
        const cd aj = a[j0 + jj], bj = b[j0 + jj];
#pragma unroll
        for (int i = 0; i < RB; ++i) {
          acc[i] = cfma(aj, xv[RB - 1 + i - jj], acc[i]);
          acc[i] = cfma(bj, yv[RB - 1 + i - jj], acc[i]);
        }
      }
    }
    if (j0 + RB < J) {
#pragma unroll
      for (int k = W - 1; k >= RB; --k) {
        xv[k] = xv[k - RB];
        yv[k] = yv[k - RB];
      }
#pragma unroll
      for (int k = 0; k < RB; ++k) {
        xv[k] = xr[skew<RB>(xo + t0 - j0 - 2 * RB + 1 + k)];
        yv[k] = yr[skew<RB>(yo + t0 - j0 - 2 * RB + 1 + k)];
      }
    }
  }
}

// sum_{j0 <= j < j1} a[j] x[-j] + b[j] y[-j] over LDS operands, unrolled by 8 so
// that the loads of a block are in flight together
__device__ __forceinline__ cd dot2(const cd* a, const cd* x, const cd* b, const cd* y, int j0,
                                   int j1) {
  cd s0{0.0, 0.0}, s1{0.0, 0.0}, s2{0.0, 0.0}, s3{0.0, 0.0};
  int j = j0;
  for (; j + 8 <= j1; j += 8) {
    cd av[8], xv[8], bv[8], yv[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      av[i] = a[j + i];
      xv[i] = x[-(j + i)];
      bv[i] = b[j + i];
      yv[i] = y[-(j + i)];
    }
#pragma unroll
    for (int i = 0; i < 8; i += 2) {
      s0 = cfma(av[i], xv[i], s0);
      s1 = cfma(bv[i], yv[i], s1);
      s2 = cfma(av[i + 1], xv[i + 1], s2);
      s3 = cfma(bv[i + 1], yv[i + 1], s3);
    }
  }
  for (; j < j1; ++j) {
    s0 = cfma(a[j], x[-j], s0);
    s1 = cfma(b[j], y[-j], s1);
  }
  return cadd(cadd(s0, s2), cadd(s1, s3));
}

// RB consecutive outputs t0.. of one polynomial of Theta2 Theta1 (shifted
// form) over the lags j < J: R[t] = sum_j q1[j] p1[t-j] + q2[j] p2[t-1-j] with
// p1, p2 the padded rows r1, r2 and origins o1, o2 (o2 already one lag back);
// the root adds the second column one more lag back (rho = R21 + z R22),
// whose rows follow at distance pe.  Writes out[0..RB).
template <int RB>
__device__ __forceinline__ void post_block(const cd* q1, const cd* r1, int o1, const cd* q2,
                                           const cd* r2, int o2, int J, int t0, bool root,
                                           int pe, cd* out) {
  cd acc[RB];
#pragma unroll
  for (int i = 0; i < RB; ++i) acc[i] = cd{0.0, 0.0};
  if (J > 0) {
    conv2_block<RB>(q1, r1, o1, q2, r2, o2, J, t0, acc);
    if (root) conv2_block<RB>(q1, r1 + pe, o1 - 1, q2, r2 + pe, o2 - 1, J, t0, acc);
  }
#pragma unroll
  for (int i = 0; i < RB; ++i) out[i] = acc[i];
}

// One Schur step on the moving window (lane r: U(n+1+r), V(n+r) at order n):
// k_n = -U(n+1)/delta_n, delta_{n+1} = delta_n (1 - |k|^2),
// V <- V + conj(k) U,  U <- (U + k V) shifted down one lane.
__device__ __forceinline__ void leaf_step(cd& U, cd& V, double& dlt, double& inv, cd& k,
                                          double& dn) {
  const cd U0 = readlane_c(U, 0);
  k = cd{-U0.x * inv, -U0.y * inv};
  const double q = 1.0 - cabs2(k);
  dn = dlt * q;
  // 1/delta_{n+1} = (1/delta_n) / q: hardware reciprocal + one Newton step
  const double r0 = __builtin_amdgcn_rcp(q);
  const double r1 = fma(r0, fma(-q, r0, 1.0), r0);
  const cd W = cfma(k, V, U);  // U(i) + k V(i-1)
  V = cfmac(U, k, V);          // V(i-1) + U(i) conj(k)
  U = shl1c(W);
  dlt = dn;
  inv = inv * r1;
}

// W_F^e = exp(-j 2 pi e / F), 0 <= e < F, from the natural-order table
__device__ __forceinline__ cd wpow(const cd* __restrict__ tw, int logtw, int e, int logF) {
  const int F = 1 << logF;
  if (e >= (F >> 1)) {
    const cd w = tw[(e - (F >> 1)) << (logtw - logF)];
    return cd{-w.x, -w.y};
  }
  return tw[e << (logtw - logF)];
}
// W_F^e for F <= FFT_TWL from the LDS copy of the stage-major table head
// (W_F^e = tws[F/2 + e] for e < F/2, and -tws[e] above)
__device__ __forceinline__ cd wpow_l(const cd* s_tw, int e, int logF) {
  const int h = 1 << (logF - 1);
  if (e >= h) {
    const cd w = s_tw[e];
    return cd{-w.x, -w.y};
  }
  return s_tw[h + e];
}
__device__ __forceinline__ cd zbin_l(const cd* s_tw, int p, int logF) {
  return wpow_l(s_tw, bitrev(p, logF), logF);
}
__device__ __forceinline__ cd row_phase_l(const cd* s_tw, int p, int logF, int m) {
  const int f = bitrev(p, logF);
  return wpow_l(s_tw, (f * (m - 1)) & ((1 << logF) - 1), logF);
}
// W_F^f for the bin at bit-reversed position p
__device__ __forceinline__ cd zbin(const cd* __restrict__ tw, int logtw, int p, int logF) {
  return wpow(tw, logtw, bitrev(p, logF), logF);
}
// Spectra of the second row of a Theta over m steps at bit-reversed bin p,
// from those of the first row (symmetry above): s21 from s12, s22 from s11,
// with ph = W_F^(f (m-1)) from row_phase.
__device__ __forceinline__ cd row_phase(const cd* __restrict__ tw, int logtw, int p, int logF,
                                        int m) {
  const int f = bitrev(p, logF);
  return wpow(tw, logtw, (f * (m - 1)) & ((1 << logF) - 1), logF);
}
__device__ __forceinline__ void second_row(cd ph, cd s11, cd s12, cd& s21, cd& s22) {
  s21 = cmul(ph, cconj(s12));
  s22 = cmul(ph, cconj(s11));
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
                                                  int64_t* __restrict__ failed,
                                                  const int32_t* __restrict__ order) {
  const int bi = order ? order[blockIdx.x] : blockIdx.x;
  if (req && !(req[bi] & REQ_EVAL)) return;
  const InstInfo in = info[bi];
  const SchurLayout& L = lay[bi];  // read through uniform addresses (scalar loads)
  const int N = in.N;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  extern __shared__ cd lds[];
  cd* A = lds;
  cd* Bf = lds + padded(L.Fmax);
  __shared__ double s_logdet;
  __shared__ int s_fail;
  __shared__ cd s_tw[FFT_TWL];  // head of the stage-major twiddle table
  const cd* cb = c + in.off;
  cd* scr = scratch + L.scr_off;
  double* dl = delta_out ? delta_out + in.off : nullptr;
  load_tw_head<SCH_NT>(s_tw, tws);
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
      // Waves 0-2 each run the m Schur steps on the window (the same code, so
      // the same coefficients); wave 0 keeps the pivots, waves 1 and 2
      // accumulate the two independent column pairs of Theta, (P11, P21) and
      // (P12, P22).
      if (wv <= 2) {
        cd U = (lane < m) ? u[lane] : cd{0.0, 0.0};
        cd V = (lane < m) ? v[lane] : cd{0.0, 0.0};
        double dlt = readlane_f64(V.x, 0);
        double inv = 1.0 / dlt;
        cd k;
        double dn;
        if (wv == 0) {
          double my_dn = 1.0;  // delta_{n0+1+lane}
          for (int s = 0; s < m; ++s) {
            leaf_step(U, V, dlt, inv, k, dn);
            if (lane == s) my_dn = dn;
          }
          // pivots, their logs and the first non-positive one, one per lane
          double lg = 0.0;
          bool bad = false;
          if (lane < m) {
            if (dl) dl[act.n0 + 1 + lane] = my_dn;
            bad = !(my_dn > 0.0) || !isfinite(my_dn);
            lg = log(my_dn);
          }
          const double lsum = wave_sum(lg);
          const unsigned long long badm = __ballot(bad);
          if (lane == 0) {
            s_logdet += lsum;
            if (badm) s_fail = act.n0 + 1 + __builtin_ctzll(badm);
          }
        } else {
          // column c = wv: after step 0 (1, conj k0) for c = 1 and (k0, 1) for
          // c = 2 (shifted form); then (P1c, P2c) <- (P1c + k z P2c, conj(k) P1c + z P2c)
          leaf_step(U, V, dlt, inv, k, dn);
          const bool l0 = lane == 0;
          const cd one{l0 ? 1.0 : 0.0, 0.0};
          const cd kk = l0 ? k : cd{0.0, 0.0};
          cd T1 = (wv == 1) ? one : kk;
          cd T2 = (wv == 1) ? cconj(kk) : one;
          for (int s = 1; s < m; ++s) {
            leaf_step(U, V, dlt, inv, k, dn);
            const cd S2 = shr1c(T2);
            const cd o1 = T1;
            T1 = cfma(k, S2, o1);
            T2 = cfmac(o1, k, S2);
          }
          if (act.type == SCH_ROOT_LEAF) {
            (wv == 1 ? A : Bf)[lane] = T2;  // P21, P22 (plain index)
          } else {
            cd* R = scr + L.res[act.level] + (int64_t)act.side * 4 * L.mmax[act.level];
            const int st = L.mmax[act.level];
            if (lane < m) {
              const int c0 = wv - 1;  // column 0 -> P11/P21, column 1 -> P12/P22
              R[c0 * st + lane] = T1;
              R[(2 + c0) * st + lane] = T2;
            }
          }
        }
      }
      __syncthreads();
      if (s_fail >= 0) break;
      if (act.type == SCH_ROOT_LEAF) {
        // rho = P21 + z P22 (degree <= m = N-1 <= 63)
        if (tid < N) rho[in.off + tid] = cadd(tid < m ? A[tid] : cd{0.0, 0.0},
                                             tid > 0 ? Bf[tid - 1] : cd{0.0, 0.0});
        __syncthreads();
      }
      continue;
    }
    const int cl = act.level + 1;
    const cd* T1 = scr + L.res[cl];              // left child's Theta (m1 coefficients each)
    const cd* T2 = T1 + (int64_t)4 * L.mmax[cl];  // right child's Theta (m2 coefficients each)
    const int st1 = L.mmax[cl];
    const bool root = act.type == SCH_ROOT;
    cd* R = scr + L.res[act.level] + (int64_t)act.side * 4 * L.mmax[act.level];
    const int st = L.mmax[act.level];
    if (m <= SCH_DIRECT) {
      if (act.type == SCH_MID) {
        // u2[r] = sum_j P11[j] u[m1+r-j] + P12[j] v[m1+r-j]
        // v2[r] = sum_j P21[j] u[m1-1+r-j] + P22[j] v[m1-1+r-j],  j < m1;
        // each sum is split in sp parts so that the block's threads share it.
        for (int t = tid; t < 4 * m1; t += SCH_NT) A[t] = T1[(t / m1) * st1 + t % m1];
        for (int t = tid; t < m; t += SCH_NT) {
          Bf[t] = u[t];
          Bf[m + t] = v[t];
        }
        __syncthreads();
        const int nout = 2 * m2;
        const int sp = nout <= SCH_NT / 4 ? 4 : (nout <= SCH_NT / 2 ? 2 : 1);
        const int jh = (m1 + sp - 1) / sp;
        cd* part = Bf + 2 * m;
        for (int it = tid; it < nout * sp; it += SCH_NT) {
          const int o = it % nout, h = it / nout;
          const bool isv = o >= m2;
          const int r = isv ? o - m2 : o;
          const cd* Pa = A + (isv ? 2 * m1 : 0);
          const cd* Pb = Pa + m1;
          const cd* xu = Bf + (isv ? m1 - 1 + r : m1 + r);
          const cd* xv = xu + m;
          const int j0 = h * jh, j1 = j0 + jh < m1 ? j0 + jh : m1;
          part[it] = dot2(Pa, xu, Pb, xv, j0, j1);
        }
        __syncthreads();
        cd* W2 = scr + L.win[cl];
        const int stw = L.mmax[cl];
        for (int o = tid; o < nout; o += SCH_NT) {
          cd acc = part[o];
          for (int h = 1; h < sp; ++h) acc = cadd(acc, part[h * nout + o]);
          const bool isv = o >= m2;
          W2[(isv ? stw + o - m2 : o)] = acc;
        }
        __syncthreads();
        continue;
      }
      // POST / ROOT in the shifted form, as sliding-window sums over j < m2
      // against zero-padded P':
      //   R11 = Q11 P11' + z Q12 P21',  R12 = Q11 P12' + z Q12 P22'
      // (the second row follows by symmetry); the root needs
      //   rho = R21 + z R22 = Q21 (P11' + z P12') + z Q22 (P21' + z P22').
      // Each sum is split in nsp parts (partials after the operands).
      const int nout = root ? N : m;   // outputs per polynomial
      const int npoly = root ? 1 : 2;
      const int RB = (npoly * nout >= 128) ? 2 : 1;
      const int lrb = RB == 2 ? 1 : 0;
      const int PL = m2 + 8;                 // zeros below each P'
      const int pe = PL + m + 8;             // padded row length (multiple-of-RB skew)
      const int pes = pe + (pe >> lrb) * (RB > 1);  // skewed row length
      cd* Pext = A;                          // row q: P'_q(i) at skew(PL + i)
      cd* Q = A + 4 * pes + 8;               // 4 x m2
      cd* part = Q + 4 * m2;
      const int nblk = (nout + RB - 1) / RB;
      const int nbr = nblk * RB;             // partial row length
      const int avail = 2 * padded(L.Fmax) - (4 * pes + 8 + 4 * m2);
      int nsp = 1;
      while (nsp < 8 && npoly * nblk * 2 * nsp <= SCH_NT && npoly * nbr * 2 * nsp <= avail)
        nsp *= 2;
      const int jl = (m2 + nsp - 1) / nsp;
      batched_for<2>(tid, SCH_NT, 4 * pe, [&](int t) {
        const int q = t / pe, i = t % pe - PL;
        return (i >= 0 && i < m1) ? T1[q * st1 + i] : cd{0.0, 0.0};
      }, [&](int t, cd v) {
        const int q = t / pe, k = t % pe;
        Pext[q * pes + (RB > 1 ? k + (k >> lrb) : k)] = v;
      });
      const int qr0 = root ? 2 : 0;          // rows of Theta2 in use
      for (int t = tid; t < 2 * m2; t += SCH_NT) Q[qr0 * m2 + t] = T2[(qr0 + t / m2) * st1 + t % m2];
      __syncthreads();
      for (int it = tid; it < npoly * nblk * nsp; it += SCH_NT) {
        const int h = it / (npoly * nblk), rem = it - h * (npoly * nblk);
        const int pl = rem / nblk, t0 = (rem - pl * nblk) * RB;
        const int col = root ? 0 : pl;
        const int j0 = h * jl, j1 = min(j0 + jl, m2);
        const cd* q1 = Q + qr0 * m2 + j0;
        const cd* q2 = q1 + m2;
        const cd* r1 = Pext + col * pes;         // P11' or P12'
        const cd* r2 = Pext + (2 + col) * pes;   // P21' or P22' (one lag)
        cd* out = part + (h * npoly + pl) * nbr + t0;
        if (RB == 2) post_block<2>(q1, r1, PL - j0, q2, r2, PL - 1 - j0, j1 - j0, t0, root, pes, out);
        else post_block<1>(q1, r1, PL - j0, q2, r2, PL - 1 - j0, j1 - j0, t0, root, pes, out);
      }
      __syncthreads();
      for (int o = tid; o < npoly * nout; o += SCH_NT) {
        const int pl = o / nout, t = o - pl * nout;
        cd acc = part[pl * nbr + t];
        for (int h = 1; h < nsp; ++h) acc = cadd(acc, part[(h * npoly + pl) * nbr + t]);
        if (root) {
          rho[in.off + t] = acc;
        } else {
          R[pl * st + t] = acc;                         // R11, R12
          R[(3 - pl) * st + (m - 1 - t)] = cconj(acc);  // R22, R21
        }
      }
      __syncthreads();
      continue;
    }
    const int logF = act.logF, F = 1 << logF;
    const double invF = 1.0 / (double)F;
    cd* S = scr + L.spec[act.level];  // spectra of Theta1's first row, 2 x F
    const int zs = pidx(F);          // buffer stride of the one-wave transforms
    if (logF <= SCH_WAVE_LOG && F <= L.ldsF && 4 * zs <= 2 * padded(L.Fmax)) {
      // One wave per transform, block barriers only around the pointwise step;
      // the spectra of Theta1's first row are transformed again by POST (in
      // waves that would idle) instead of kept in scratch between the two.
      cd* Z = lds;
      if (act.type == SCH_MID) {
        // waves 0-3: spectra of P11, P12 and of the window u, v
        if (wv < 4) {
          const cd* src = wv == 0 ? T1 : (wv == 1 ? T1 + st1 : (wv == 2 ? u : v));
          const int lim = wv < 2 ? m1 : m;
          cd* z = Z + wv * zs;
          batched_for<8>(lane, 64, F, [&](int t) { return t < lim ? src[t] : cd{0.0, 0.0}; },
                         [&](int t, cd x) { z[pidx(t)] = x; });
          wave_sync();
          wave_dif(z, logF, false, s_tw, tws, lane);
        }
        __syncthreads();
        batched_for<2>(tid, SCH_NT, F, [&](int p) { return row_phase_l(s_tw, p, logF, m1); },
                       [&](int p, cd ph) {
          const cd s11 = Z[pidx(p)], s12 = Z[zs + pidx(p)];
          const cd fu = Z[2 * zs + pidx(p)], fv = Z[3 * zs + pidx(p)];
          cd s21, s22;
          second_row(ph, s11, s12, s21, s22);
          Z[2 * zs + pidx(p)] = cfma(s12, fv, cmul(s11, fu));
          Z[3 * zs + pidx(p)] = cfma(s22, fv, cmul(s21, fu));
        });
        __syncthreads();
        // waves 2, 3: P1 and P2, and from them the right child's window
        if (wv == 2 || wv == 3) {
          cd* z = Z + wv * zs;
          wave_dit(z, logF, true, s_tw, tws, lane);
          cd* W2 = scr + L.win[cl] + (wv == 3 ? L.mmax[cl] : 0);
          const int o = wv == 2 ? m1 : m1 - 1;
          for (int r = lane; r < m2; r += 64) W2[r] = cscale(z[pidx(o + r)], invF);
        }
        __syncthreads();
        continue;
      }
      // POST / ROOT (one row as below): waves 0, 1 transform the row of
      // Theta2, waves 2, 3 the first row of Theta1 (P11, P12)
      const int row = root ? 1 : 0;
      if (wv < 4) {
        const cd* src = wv < 2 ? T2 + (2 * row + wv) * st1 : T1 + (wv - 2) * st1;
        const int lim = wv < 2 ? m2 : m1;
        cd* z = Z + wv * zs;
        batched_for<8>(lane, 64, F, [&](int t) { return t < lim ? src[t] : cd{0.0, 0.0}; },
                       [&](int t, cd x) { z[pidx(t)] = x; });
        wave_sync();
        wave_dif(z, logF, false, s_tw, tws, lane);
      }
      __syncthreads();
      batched_for<2>(tid, SCH_NT, F, [&](int p) {
        return cd2{zbin_l(s_tw, p, logF), row_phase_l(s_tw, p, logF, m1)};
      }, [&](int p, cd2 g) {
        const cd zb = g.a;
        const cd a1 = Z[pidx(p)], a2 = cmul(Z[zs + pidx(p)], zb);
        const cd s11 = Z[2 * zs + pidx(p)], s12 = Z[3 * zs + pidx(p)];
        cd s21, s22;
        second_row(g.b, s11, s12, s21, s22);
        const cd r1 = cfma(a2, s21, cmul(a1, s11));
        const cd r2 = cfma(a2, s22, cmul(a1, s12));
        if (root) {
          Z[pidx(p)] = cfma(r2, zb, r1);
        } else {
          Z[pidx(p)] = r1;
          Z[zs + pidx(p)] = r2;
        }
      });
      __syncthreads();
      if (root) {
        if (wv == 0) {
          wave_dit(Z, logF, true, s_tw, tws, lane);
          for (int t = lane; t < N; t += 64) rho[in.off + t] = cscale(Z[pidx(t)], invF);
        }
      } else if (wv < 2) {
        // wave 0: R11 and R22; wave 1: R12 and R21
        cd* z = Z + wv * zs;
        wave_dit(z, logF, true, s_tw, tws, lane);
        for (int t = lane; t < m; t += 64) {
          const cd r = cscale(z[pidx(t)], invF);
          R[wv * st + t] = r;
          R[(3 - wv) * st + (m - 1 - t)] = cconj(r);
        }
      }
      __syncthreads();
      continue;
    }
    // Transform buffers: LDS, or for F > L.ldsF two buffers in the
    // instance's scratch (the same passes, on global memory).
    auto fft_merge = [&](cd* __restrict__ A, cd* __restrict__ Bf) __attribute__((always_inline)) {
      if (act.type == SCH_MID) {
        // job 0: spectra of P11 and P12 (to S); job 1: the window
        for (int job = 0; job < 2; ++job) {
          const cd* pa = job == 0 ? T1 : u;
          const cd* pb = job == 0 ? T1 + st1 : v;
          const int lim = job == 0 ? m1 : m;
          batched_for<4>(tid, SCH_NT, F, [&](int t) {
            return t < lim ? cd2{pa[t], pb[t]} : cd2{cd{0.0, 0.0}, cd{0.0, 0.0}};
          }, [&](int t, cd2 x) {
            A[pidx(t)] = x.a;
            Bf[pidx(t)] = x.b;
          });
          __syncthreads();
          dif_fftn<SCH_NT>(A, Bf, 2, logF, false, false, s_tw, tws);
          if (job == 0) {
            for (int t = tid; t < F; t += SCH_NT) {
              S[t] = A[pidx(t)];
              S[F + t] = Bf[pidx(t)];
            }
            __syncthreads();
          }
        }
        batched_for<4>(tid, SCH_NT, F, [&](int p) {
          return cd4{row_phase(tw, logtw, p, logF, m1), S[p], S[F + p], cd{0.0, 0.0}};
        }, [&](int p, cd4 g) {
          const cd fu = A[pidx(p)], fv = Bf[pidx(p)];
          const cd s11 = g.b, s12 = g.c;
          cd s21, s22;
          second_row(g.a, s11, s12, s21, s22);
          A[pidx(p)] = cfma(s12, fv, cmul(s11, fu));
          Bf[pidx(p)] = cfma(s22, fv, cmul(s21, fu));
        });
        __syncthreads();
        dit_fftn<SCH_NT>(A, Bf, 2, logF, true, true, s_tw, tws);
        // right child's window
        cd* W2 = scr + L.win[cl];
        const int stw = L.mmax[cl];
        for (int r = tid; r < m2; r += SCH_NT) {
          W2[r] = cscale(A[pidx(m1 + r)], invF);
          W2[stw + r] = cscale(Bf[pidx(m1 - 1 + r)], invF);
        }
        __syncthreads();
        return;
      }
      // POST / ROOT: one row of Theta = Theta2 Theta1, the first (the second
      // follows by symmetry), or for the root the second, whose
      // rho = R21 + z R22.
      const int row = root ? 1 : 0;
      batched_for<4>(tid, SCH_NT, F, [&](int t) {
        return (t < m2) ? cd2{T2[(2 * row) * st1 + t], T2[(2 * row + 1) * st1 + t]}
                        : cd2{cd{0.0, 0.0}, cd{0.0, 0.0}};
      }, [&](int t, cd2 x) {
        A[pidx(t)] = x.a;
        Bf[pidx(t)] = x.b;
      });
      __syncthreads();
      dif_fftn<SCH_NT>(A, Bf, 2, logF, false, false, s_tw, tws);
      batched_for<4>(tid, SCH_NT, F, [&](int p) {
        return cd4{zbin(tw, logtw, p, logF), row_phase(tw, logtw, p, logF, m1), S[p], S[F + p]};
      }, [&](int p, cd4 g) {
        const cd zb = g.a;
        const cd a1 = A[pidx(p)], a2 = cmul(Bf[pidx(p)], zb);  // z * second poly
        const cd s11 = g.c, s12 = g.d;
        cd s21, s22;
        second_row(g.b, s11, s12, s21, s22);
        const cd r1 = cfma(a2, s21, cmul(a1, s11));   // row . column 1
        const cd r2 = cfma(a2, s22, cmul(a1, s12));   // row . column 2 (shifted)
        if (root) {
          A[pidx(p)] = cfma(r2, zb, r1);  // rho = R21 + z R22'
        } else {
          A[pidx(p)] = r1;
          Bf[pidx(p)] = r2;
        }
      });
      __syncthreads();
      dit_fftn<SCH_NT>(A, Bf, root ? 1 : 2, logF, true, true, s_tw, tws);
      if (root) {
        for (int t = tid; t < N; t += SCH_NT) rho[in.off + t] = cscale(A[pidx(t)], invF);
      } else {
        for (int t = tid; t < m; t += SCH_NT) {
          const cd r11 = cscale(A[pidx(t)], invF), r12 = cscale(Bf[pidx(t)], invF);
          R[t] = r11;
          R[st + t] = r12;
          R[2 * st + (m - 1 - t)] = cconj(r12);
          R[3 * st + (m - 1 - t)] = cconj(r11);
        }
      }
      __syncthreads();
    };
    if (F > L.ldsF) fft_merge(scr + L.xbig, scr + L.xbig + padded(F));
    else fft_merge(lds, lds + padded(L.Fmax));
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
                        int B, int Fmax, hipStream_t st, const int32_t* order) {
  const size_t shm = 2 * (size_t)padded(Fmax) * sizeof(cd);
  (void)hipFuncSetAttribute((const void*)k_schur, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)shm);
  hipLaunchKernelGGL(k_schur, dim3(B), dim3(SCH_NT), shm, st, info, req, lay, acts, c, tw, logtw,
                     tws, scratch, rho, delta, logdet, status, failed, order);
  return hipGetLastError();
}

}  // namespace sfls
