// Incomplete observations (Sec. IV): the evaluation of the estimator's
// objective when Phi keeps M weighted samples of N, by the semifast method.
//
// With A = Phi Psi(theta), Gamma^{1/2} = diag(sqrt gamma) and
// K_s = beta I + Gamma^{1/2} A^H A Gamma^{1/2} = L L^H (K x K, positive
// definite for beta > 0 whatever gamma >= 0), Woodbury's identity (the
// scaled form of eq. CfromSigma) and the matrix determinant lemma give
//   C^{-1}     = beta^{-1} (I - A Gamma^{1/2} K_s^{-1} Gamma^{1/2} A^H)
//   ln|C|      = (M - K) ln beta + 2 sum_k ln L_kk
//   C^{-1} y   = (y - A c) / beta,  c = Gamma^{1/2} K_s^{-1} Gamma^{1/2} A^H y
// and with the Gram matrices G_p = A^H D^p A (eq. AhA and its D-weighted
// forms, D = diag(2 pi n_m)), Z_p = L^{-1} Gamma^{1/2} G_p, e_k = L^{-1} e_k:
//   s_k = (G0_kk - |Z0_k|^2) / beta      t_k = (G1_kk - Z1_k^H Z0_k) / beta
//   v_k = (G2_kk - Z2_k^H Z0_k) / beta   x_k = (G2_kk - |Z1_k|^2) / beta
// (eqs. s, t, v, x).  For a component whose posterior variance is well below
// its prior (beta [K_s^{-1}]_kk < 1/2) the first three are taken in the
// equivalent product form gamma_k^{-1/2} Z_p_k^H e_k, which avoids the
// cancellation of the difference form there.  q, r, u (eqs. q, r, u) are the
// direct sums of Psi^H D^p Phi^H C^{-1} y over the observed samples.
//
// Grid sweeps (Sec. IV, "q and s at all gridpoints"): Phi^H C^{-1} y is
// scattered into an N-vector for the grid transform of q^G, and
//   E = Phi^H C^{-1} Phi = beta^{-1} (Phi^H Phi - U U^H),
//   U = Phi^H A Gamma^{1/2} L^{-H}  (N x K, nonzero on the observed rows),
// so the diagonal sums omega_s(i) of E are beta^{-1} (sum |phi|^2 [i = 0] -
// sum_j sum_n U_nj conj(U_{n+i,j})): one autocorrelation per column of U by
// P-point transforms (P >= 2N - 1), which the grid stage turns into s^G as
// for complete data.  At candidate frequencies q and s are direct sums:
// s(theta) = beta^{-1} (sum |phi|^2 - sum_j |psi(theta)^H U_j|^2).
#include "sfls_kernels.hpp"
#include "k_launch.hpp"

namespace sfls {

constexpr int SF_NT = 256;
constexpr int SFG_NT = 512;  // Gram sums
constexpr int SF_MT = 64;    // rows of A staged per chunk of the Gram sums
constexpr int SF_KP = SF_KMAX + 2;  // staged row length (columns 0..K, a zero pad)
constexpr int SF_UMT = 64;   // rows per chunk of the grid columns U
constexpr int SF_CANDB = 8;  // blocks per instance of the candidate sums

__device__ __forceinline__ cd sf_phi(const cd* __restrict__ phi, int64_t i) {
  return phi ? phi[i] : cd{1.0, 0.0};
}
template <typename YT>
__device__ __forceinline__ cd sf_y(const YT* __restrict__ y, int64_t i) {
  return cd{(double)y[i].x, (double)y[i].y};
}
// An instance's block of 4 kcap x kcap matrices at sfoff: G_0, G_1, G_2
// (column-major), then L^{-1} (row-major).
__device__ __forceinline__ int64_t sf_g(const InstInfo& in, int p, int i, int k) {
  return in.sfoff + (int64_t)p * in.kcap * in.kcap + (int64_t)k * in.kcap + i;
}
__device__ __forceinline__ int64_t sf_li(const InstInfo& in, int i, int k) {
  return in.sfoff + (int64_t)3 * in.kcap * in.kcap + (int64_t)i * in.kcap + k;
}
// e^{j 2 pi n theta_k} from component k's phase tables (tb: the instance's tables)
__device__ __forceinline__ cd sf_cis(const cd* __restrict__ tb, int W, int B1, int k, int n) {
  const cd* t = tb + (int64_t)k * W;
  return cmul(t[n >> 6], t[B1 + (n & 63)]);
}

// ---------------------------------------------------------------------------
// Phase tables of the evaluation point's components (REQ_EVAL).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(SF_NT) void k_sf_tables(const InstInfo* __restrict__ info,
                                                     const int32_t* __restrict__ req,
                                                     const int32_t* __restrict__ Kev,
                                                     const double* __restrict__ theta,
                                                     cd* __restrict__ tabs) {
  const int b = blockIdx.x;
  if (!(req[b] & REQ_EVAL)) return;
  const InstInfo in = info[b];
  const int K = Kev[b], B1 = SF_TB1(in.N), W = SF_TBW(in.N);
  cd* tb = tabs + in.tboff;
  for (int e = threadIdx.x; e < K * W; e += SF_NT) {
    const int k = e / W, j = e % W;
    const double n = j < B1 ? 64.0 * (double)j : (double)(j - B1);
    tb[e] = cis2pi(frac_mul(n, theta[in.koff + k]));
  }
}

// ---------------------------------------------------------------------------
// Gram sums.  The columns of A are augmented by y (column K), so that the
// last column of G0 is h = A^H y.  Each thread accumulates a 2 x 2 tile of the
// upper triangle of the three weighted sums over its slice of the rows; the
// slices are summed in a fixed order.  The rows of a chunk (index, weight,
// sample) are staged in LDS once, their A entries from the phase tables.
// ---------------------------------------------------------------------------
template <typename YT>
__global__ __launch_bounds__(SFG_NT) void k_sf_gram(const InstInfo* __restrict__ info,
                                                    const int32_t* __restrict__ req,
                                                    const int32_t* __restrict__ Kev,
                                                    const cd* __restrict__ tabs,
                                                    const YT* __restrict__ y,
                                                    const int32_t* __restrict__ idx,
                                                    const cd* __restrict__ phi,
                                                    cd* __restrict__ sfm, cd* __restrict__ h) {
  const int b = blockIdx.x;
  if (!(req[b] & REQ_EVAL)) return;
  const InstInfo in = info[b];
  const int K = Kev[b];
  if (K <= 0) return;
  const int M = in.nobs;
  const int Kc = K + 1;
  const int nb = (Kc + 1) / 2;
  const int ntile = nb * (nb + 1) / 2;
  const int tid = threadIdx.x;
  const int B1 = SF_TB1(in.N), W = SF_TBW(in.N);
  const cd* tb = tabs + in.tboff;
  // LDS: the staged rows (SF_MT x SF_KP), their weights 2 pi n, indices,
  // phi and y; reused for the slice partials (SFG_NT x 12)
  extern __shared__ cd sf_lds[];
  cd* sP = sf_lds;
  double* sd = reinterpret_cast<double*>(sP + SF_MT * SF_KP);
  int32_t* sn = reinterpret_cast<int32_t*>(sd + SF_MT);
  cd* sph = reinterpret_cast<cd*>(sn + SF_MT);
  cd* sy = sph + SF_MT;
  const int S = ntile >= SFG_NT ? 1 : min(16, SFG_NT / ntile);
  const int npass = S == 1 ? (ntile + SFG_NT - 1) / SFG_NT : 1;
  const int64_t mo = in.obsoff;
  for (int pass = 0; pass < npass; ++pass) {
    int tile, slice;
    if (S == 1) { tile = pass * SFG_NT + tid; slice = 0; }
    else { tile = tid % ntile; slice = tid / ntile; }
    const bool act = tile < ntile && slice < S;
    int bi = 0, bk = 0;
    if (act) {
      int t = tile;
      while (t >= nb - bi) { t -= nb - bi; ++bi; }
      bk = bi + t;
    }
    const int i0 = 2 * bi, k0 = 2 * bk;
    cd acc[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) acc[q] = cd{0.0, 0.0};
    for (int m0 = 0; m0 < M; m0 += SF_MT) {
      const int rows = min(SF_MT, M - m0);
      __syncthreads();
      if (tid < rows) {
        const int64_t m = mo + m0 + tid;
        const int32_t n = idx[m];
        sn[tid] = n;
        sd[tid] = 2.0 * M_PI * (double)n;
        sph[tid] = sf_phi(phi, m);
        sy[tid] = sf_y(y, m);
      }
      __syncthreads();
      for (int e = tid; e < rows * (Kc + 1); e += SFG_NT) {
        const int r = e / (Kc + 1), k = e % (Kc + 1);
        cd v{0.0, 0.0};
        if (k < K) v = cmul(sph[r], sf_cis(tb, W, B1, k, sn[r]));
        else if (k == K) v = sy[r];
        sP[r * SF_KP + k] = v;
      }
      __syncthreads();
      if (act) {
        for (int r = slice; r < rows; r += S) {
          const cd* row = sP + r * SF_KP;
          const cd a = row[i0], bb = row[i0 + 1], c = row[k0], d = row[k0 + 1];
          const double w = sd[r], w2 = w * w;
          const cd p[4] = {cmulc(c, a), cmulc(d, a), cmulc(c, bb), cmulc(d, bb)};  // conj(x) y
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            acc[q] = cadd(acc[q], p[q]);
            acc[4 + q].x = fma(w, p[q].x, acc[4 + q].x);
            acc[4 + q].y = fma(w, p[q].y, acc[4 + q].y);
            acc[8 + q].x = fma(w2, p[q].x, acc[8 + q].x);
            acc[8 + q].y = fma(w2, p[q].y, acc[8 + q].y);
          }
        }
      }
    }
    if (S > 1) {
      __syncthreads();
      if (act) {
#pragma unroll
        for (int q = 0; q < 12; ++q) sf_lds[tid * 12 + q] = acc[q];
      }
      __syncthreads();
      if (act && slice == 0) {
        for (int s = 1; s < S; ++s) {
#pragma unroll
          for (int q = 0; q < 12; ++q) acc[q] = cadd(acc[q], sf_lds[(s * ntile + tile) * 12 + q]);
        }
      }
    }
    if (act && slice == 0) {
#pragma unroll
      for (int di = 0; di < 2; ++di)
#pragma unroll
        for (int dk = 0; dk < 2; ++dk) {
          const int i = i0 + di, k = k0 + dk;
          if (i > k || i >= K || k > K) continue;
          const int q = 2 * di + dk;
          if (k == K) {
            h[in.koff + i] = acc[q];
            continue;
          }
#pragma unroll
          for (int p = 0; p < 3; ++p) {
            cd v = acc[4 * p + q];
            if (i == k) v.y = 0.0;
            sfm[sf_g(in, p, i, k)] = v;
            if (i != k) sfm[sf_g(in, p, k, i)] = cconj(v);
          }
        }
    }
  }
}
// LDS of k_sf_gram: the staged rows and row data, or the slice partials
constexpr size_t SFG_LDS_ROWS = (size_t)SF_MT * SF_KP * sizeof(cd) + SF_MT * (sizeof(double) +
                                sizeof(int32_t) + 2 * sizeof(cd));
constexpr size_t SFG_LDS = SFG_LDS_ROWS > (size_t)SFG_NT * 12 * sizeof(cd)
                               ? SFG_LDS_ROWS : (size_t)SFG_NT * 12 * sizeof(cd);

// ---------------------------------------------------------------------------
// Cholesky of K_s in LDS, L^{-1}, the active-set vectors s, t, v, x, the
// coefficients c and ln|C|.
// ---------------------------------------------------------------------------
constexpr int SF_LDK = SF_KMAX + 1;  // LDS row stride of the K x K matrices

__global__ __launch_bounds__(SF_NT) void k_sf_solve(const InstInfo* __restrict__ info,
                                                    const int32_t* __restrict__ req,
                                                    const int32_t* __restrict__ Kev,
                                                    const double* __restrict__ gamma,
                                                    const double* __restrict__ beta,
                                                    cd* __restrict__ sfm,
                                                    const cd* __restrict__ h,
                                                    cd* __restrict__ cvec,
                                                    cd* __restrict__ os, cd* __restrict__ ot,
                                                    cd* __restrict__ ov, cd* __restrict__ ox,
                                                    double* __restrict__ logdet,
                                                    int32_t* __restrict__ status) {
  const int b = blockIdx.x;
  if (!(req[b] & REQ_EVAL)) return;
  const InstInfo in = info[b];
  const int K = Kev[b];
  const int M = in.nobs;
  const double be = beta[b];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  extern __shared__ cd sf_lds[];
  cd* Ls = sf_lds;                       // K_s, then its Cholesky factor (lower)
  cd* Li = sf_lds + SF_KMAX * SF_LDK;    // L^{-1} (lower)
  __shared__ double sg[SF_KMAX];
  __shared__ cd su[SF_KMAX];
  __shared__ int s_bad;
  if (K <= 0) {
    if (tid == 0) {
      logdet[b] = (double)M * log(be);
      status[b] = 0;
    }
    return;
  }
  const double* ga = gamma + in.koff;
  for (int k = tid; k < K; k += SF_NT) sg[k] = sqrt(fmax(ga[k], 0.0));
  if (tid == 0) s_bad = 0;
  __syncthreads();
  for (int e = tid; e < K * K; e += SF_NT) {
    const int i = e / K, k = e % K;
    if (k > i) continue;
    cd v = sfm[sf_g(in, 0, i, k)];
    v.x *= sg[i] * sg[k];
    v.y *= sg[i] * sg[k];
    if (i == k) { v.x += be; v.y = 0.0; }
    Ls[i * SF_LDK + k] = v;
  }
  __syncthreads();
  // right-looking Cholesky, one column per step
  for (int j = 0; j < K; ++j) {
    const double d = Ls[j * SF_LDK + j].x;
    if (!(d > 0.0) || !isfinite(d)) {
      if (tid == 0) s_bad = 1;
      break;
    }
    const double ljj = sqrt(d), inv = 1.0 / ljj;
    for (int i = j + 1 + tid; i < K; i += SF_NT) {
      cd v = Ls[i * SF_LDK + j];
      Ls[i * SF_LDK + j] = cd{v.x * inv, v.y * inv};
    }
    __syncthreads();
    if (tid == 0) Ls[j * SF_LDK + j] = cd{ljj, 0.0};
    const int r = K - j - 1;
    for (int e = tid; e < r * r; e += SF_NT) {
      const int i = j + 1 + e / r, k = j + 1 + e % r;
      if (k > i) continue;
      const cd a = Ls[i * SF_LDK + j], c = Ls[k * SF_LDK + j];
      Ls[i * SF_LDK + k] = csub(Ls[i * SF_LDK + k], cmulc(a, c));  // L_ij conj(L_kj)
    }
    __syncthreads();
  }
  __syncthreads();
  if (s_bad) {
    if (tid == 0) status[b] = -4;  // SFLS_ENOTPD: K_s not positive definite
    return;
  }
  // L^{-1}, one column per thread: forward substitution on e_j
  for (int j = tid; j < K; j += SF_NT) {
    Li[j * SF_LDK + j] = cd{1.0 / Ls[j * SF_LDK + j].x, 0.0};
    for (int i = j + 1; i < K; ++i) {
      cd acc{0.0, 0.0};
      for (int l = j; l < i; ++l) acc = cfma(Ls[i * SF_LDK + l], Li[l * SF_LDK + j], acc);
      const double rd = -1.0 / Ls[i * SF_LDK + i].x;
      Li[i * SF_LDK + j] = cd{acc.x * rd, acc.y * rd};
    }
  }
  __syncthreads();
  for (int e = tid; e < K * K; e += SF_NT) {
    const int i = e / K, k = e % K;
    sfm[sf_li(in, i, k)] = (k <= i) ? Li[i * SF_LDK + k] : cd{0.0, 0.0};
  }
  // s, t, v, x of component k: one wave per component, row i on lane i
  for (int k = wv; k < K; k += SF_NT / 64) {
    const int i = lane;
    cd z0{0.0, 0.0}, z1{0.0, 0.0}, z2{0.0, 0.0}, ek{0.0, 0.0};
    if (i < K) {
      for (int l = 0; l <= i; ++l) {
        const cd li = Li[i * SF_LDK + l];
        const cd f = cd{li.x * sg[l], li.y * sg[l]};
        z0 = cfma(f, sfm[sf_g(in, 0, l, k)], z0);
        z1 = cfma(f, sfm[sf_g(in, 1, l, k)], z1);
        z2 = cfma(f, sfm[sf_g(in, 2, l, k)], z2);
      }
      if (k <= i) ek = Li[i * SF_LDK + k];
    }
    // z_a^H z_b and z_a^H e terms
    const cd z00 = cmulc(z0, z0), z10 = cmulc(z0, z1), z20 = cmulc(z0, z2), z11 = cmulc(z1, z1);
    const cd z0e = cmulc(ek, z0), z1e = cmulc(ek, z1), z2e = cmulc(ek, z2);
    const double s00 = wave_sum(z00.x), s11 = wave_sum(z11.x), see = wave_sum(cabs2(ek));
    const cd s10 = wave_sum(z10), s20 = wave_sum(z20);
    const double p0 = wave_sum(z0e.x);
    const cd p1 = wave_sum(z1e), p2 = wave_sum(z2e);
    if (lane == 0) {
      const double g0 = sfm[sf_g(in, 0, k, k)].x;
      const cd g1 = sfm[sf_g(in, 1, k, k)], g2 = sfm[sf_g(in, 2, k, k)];
      const double ib = 1.0 / be;
      const bool strong = sg[k] > 0.0 && be * see < 0.5;
      cd s, t, v;
      if (strong) {
        const double is = 1.0 / sg[k];
        s = cd{p0 * is, 0.0};
        t = cd{p1.x * is, p1.y * is};
        v = cd{p2.x * is, p2.y * is};
      } else {
        s = cd{(g0 - s00) * ib, 0.0};
        t = cd{(g1.x - s10.x) * ib, (g1.y - s10.y) * ib};
        v = cd{(g2.x - s20.x) * ib, (g2.y - s20.y) * ib};
      }
      os[in.koff + k] = s;
      ot[in.koff + k] = t;
      ov[in.koff + k] = v;
      ox[in.koff + k] = cd{(g2.x - s11) * ib, 0.0};
    }
  }
  // c = Gamma^{1/2} L^{-H} L^{-1} Gamma^{1/2} h, and ln|C|
  if (wv == 0) {
    const cd* hb = h + in.koff;
    cd u{0.0, 0.0};
    if (lane < K)
      for (int l = 0; l <= lane; ++l) {
        const cd li = Li[lane * SF_LDK + l];
        u = cfma(cd{li.x * sg[l], li.y * sg[l]}, hb[l], u);
      }
    if (lane < K) su[lane] = u;
    wave_sync();
    cd c{0.0, 0.0};
    if (lane < K) {
      for (int i = lane; i < K; ++i) c = cfma(cconj(Li[i * SF_LDK + lane]), su[i], c);
      cvec[in.koff + lane] = cd{c.x * sg[lane], c.y * sg[lane]};
    }
    double ld = lane < K ? 2.0 * log(Ls[lane * SF_LDK + lane].x) : 0.0;
    ld = wave_sum(ld);
    if (lane == 0) {
      logdet[b] = (double)(M - K) * log(be) + ld;
      status[b] = 0;
    }
  }
}

// ---------------------------------------------------------------------------
// C^{-1} y = (y - A c) / beta over the observed samples, y^H C^{-1} y,
// ||C^{-1} y||^2, and q, r, u (eqs. q, r, u).
// ---------------------------------------------------------------------------
template <typename YT>
__global__ __launch_bounds__(SF_NT) void k_sf_resid(const InstInfo* __restrict__ info,
                                                    const int32_t* __restrict__ req,
                                                    const int32_t* __restrict__ Kev,
                                                    const double* __restrict__ theta,
                                                    const double* __restrict__ beta,
                                                    const YT* __restrict__ y,
                                                    const int32_t* __restrict__ idx,
                                                    const cd* __restrict__ phi,
                                                    const cd* __restrict__ tabs,
                                                    const cd* __restrict__ cvec,
                                                    const int32_t* __restrict__ status,
                                                    cd* __restrict__ wM, double* __restrict__ yCy,
                                                    double* __restrict__ ww, cd* __restrict__ oq,
                                                    cd* __restrict__ orr, cd* __restrict__ ou) {
  const int b = blockIdx.x;
  if (!(req[b] & REQ_EVAL) || status[b] != 0) return;
  const InstInfo in = info[b];
  const int K = Kev[b];
  const int M = in.nobs;
  const double ib = 1.0 / beta[b];
  const int tid = threadIdx.x;
  const int B1 = SF_TB1(in.N), W = SF_TBW(in.N);
  const cd* tb = tabs + in.tboff;
  __shared__ cd sc[SF_KMAX];
  __shared__ double red[48 * (SF_NT / 64)];
  for (int k = tid; k < K; k += SF_NT) sc[k] = cvec[in.koff + k];
  __syncthreads();
  const int64_t mo = in.obsoff;
  double a2[2] = {0.0, 0.0};
  for (int m = tid; m < M; m += SF_NT) {
    const int ni = idx[mo + m];
    cd pc{0.0, 0.0};
    for (int k = 0; k < K; ++k) pc = cfma(sf_cis(tb, W, B1, k, ni), sc[k], pc);
    pc = cmul(sf_phi(phi, mo + m), pc);
    const cd ym = sf_y(y, mo + m);
    const cd wm = cd{(ym.x - pc.x) * ib, (ym.y - pc.y) * ib};
    wM[mo + m] = wm;
    a2[0] = fma(ym.x, wm.x, fma(ym.y, wm.y, a2[0]));  // Re(conj(y) w)
    a2[1] = fma(wm.x, wm.x, fma(wm.y, wm.y, a2[1]));
  }
  block_sum<SF_NT, 2>(a2, red);
  if (tid == 0) {
    yCy[b] = a2[0];
    ww[b] = a2[1];
  }
  // q, r, u in chunks of 8 components
  for (int k0 = 0; k0 < K; k0 += 8) {
    double acc[48];
#pragma unroll
    for (int q = 0; q < 48; ++q) acc[q] = 0.0;
    for (int m = tid; m < M; m += SF_NT) {
      const int ni = idx[mo + m];
      const cd v = cmulc(wM[mo + m], sf_phi(phi, mo + m));  // conj(phi) w
      const double d = 2.0 * M_PI * (double)ni;
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        if (k0 + kk >= K) break;
        const cd t = cmulc(v, sf_cis(tb, W, B1, k0 + kk, ni));  // e^{-j...} conj(phi) w
        acc[6 * kk + 0] += t.x;
        acc[6 * kk + 1] += t.y;
        acc[6 * kk + 2] = fma(d, t.x, acc[6 * kk + 2]);
        acc[6 * kk + 3] = fma(d, t.y, acc[6 * kk + 3]);
        acc[6 * kk + 4] = fma(d * d, t.x, acc[6 * kk + 4]);
        acc[6 * kk + 5] = fma(d * d, t.y, acc[6 * kk + 5]);
      }
    }
    block_sum<SF_NT, 48>(acc, red);
    if (tid < 8 && k0 + tid < K) {
      const int k = k0 + tid;
      double v6[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) v6[q] = acc[6 * 0 + q];
      // each of the 8 threads picks its component's sums
#pragma unroll
      for (int kk = 1; kk < 8; ++kk)
        if (tid == kk)
#pragma unroll
          for (int q = 0; q < 6; ++q) v6[q] = acc[6 * kk + q];
      oq[in.koff + k] = cd{v6[0], v6[1]};
      orr[in.koff + k] = cd{v6[2], v6[3]};
      ou[in.koff + k] = cd{v6[4], v6[5]};
    }
  }
}

// ---------------------------------------------------------------------------
// Grid stage inputs: w = Phi^H C^{-1} y as an N-vector (each sample found by
// a binary search of the observed indices, so every entry is written once),
// and the columns U_j (column-major, nobs x kcap) as a small product of the
// staged rows of A Gamma^{1/2} with L^{-H}.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(SF_NT) void k_sf_prep(const InstInfo* __restrict__ info,
                                                   const int32_t* __restrict__ req,
                                                   const int32_t* __restrict__ Kev,
                                                   const double* __restrict__ theta,
                                                   const double* __restrict__ gamma,
                                                   const int32_t* __restrict__ idx,
                                                   const cd* __restrict__ phi,
                                                   const cd* __restrict__ wM,
                                                   const cd* __restrict__ sfm,
                                                   const cd* __restrict__ tabs,
                                                   cd* __restrict__ w, cd* __restrict__ U) {
  const int b = blockIdx.x;
  if (!(req[b] & REQ_GRID)) return;
  const InstInfo in = info[b];
  const int K = Kev[b], M = in.nobs, N = in.N;
  const int64_t mo = in.obsoff;
  const int tid = threadIdx.x;
  // observed sample m writes its entry and zeroes the gap below it (the
  // indices increase), the last one also the gap above: each entry once
  cd* wb = w + in.off;
  for (int m = tid; m < M; m += SF_NT) {
    const int n = idx[mo + m];
    const int lo = m > 0 ? idx[mo + m - 1] + 1 : 0;
    for (int z = lo; z < n; ++z) wb[z] = cd{0.0, 0.0};
    wb[n] = cmulc(wM[mo + m], sf_phi(phi, mo + m));
    if (m == M - 1)
      for (int z = n + 1; z < N; ++z) wb[z] = cd{0.0, 0.0};
  }
  if (K <= 0) return;
  const int B1 = SF_TB1(N), W = SF_TBW(N);
  const cd* tb = tabs + in.tboff;
  extern __shared__ cd sf_lds[];
  cd* sE = sf_lds;                      // SF_UMT x SF_LDK: |phi|^2 e^{j 2pi n theta_k} sqrt(gamma_k)
  cd* sW = sf_lds + SF_UMT * SF_LDK;    // K x SF_LDK: W[k][j] = conj(L^{-1}[j][k])
  __shared__ double sg[SF_KMAX];
  for (int k = tid; k < K; k += SF_NT) sg[k] = sqrt(fmax(gamma[in.koff + k], 0.0));
  for (int e = tid; e < K * K; e += SF_NT) {
    const int k = e / K, j = e % K;
    sW[k * SF_LDK + j] = cconj(sfm[sf_li(in, j, k)]);
  }
  cd* Ub = U + in.uoff;
  for (int m0 = 0; m0 < M; m0 += SF_UMT) {
    const int rows = min(SF_UMT, M - m0);
    __syncthreads();
    for (int e = tid; e < rows * K; e += SF_NT) {
      const int r = e / K, k = e % K;
      const int64_t m = mo + m0 + r;
      const double p2 = phi ? cabs2(phi[m]) : 1.0;
      const cd ev = sf_cis(tb, W, B1, k, idx[m]);
      sE[r * SF_LDK + k] = cd{ev.x * p2 * sg[k], ev.y * p2 * sg[k]};
    }
    __syncthreads();
    for (int e = tid; e < rows * K; e += SF_NT) {
      const int j = e / rows, r = e % rows;  // consecutive threads: consecutive rows of column j
      cd acc{0.0, 0.0};
      for (int k = 0; k <= j; ++k) acc = cfma(sE[r * SF_LDK + k], sW[k * SF_LDK + j], acc);
      Ub[(int64_t)j * M + m0 + r] = acc;
    }
  }
}

// ---------------------------------------------------------------------------
// omega_s from the autocorrelations of the columns of U (P-point transforms
// in LDS, or for P > CONV_LDS_P in the instance's scratch after its first P
// block, which holds the running sum of |FFT(U_j)|^2).  Output as the grid
// stage reads it: lag i at index i mod P of oms (P points at poff).
// ---------------------------------------------------------------------------
constexpr int SFO_NT = 512;

__global__ __launch_bounds__(SFO_NT) void k_sf_omega(const InstInfo* __restrict__ info,
                                                     const int32_t* __restrict__ req,
                                                     const int32_t* __restrict__ Kev,
                                                     const double* __restrict__ beta,
                                                     const int32_t* __restrict__ idx,
                                                     const cd* __restrict__ phi,
                                                     const cd* __restrict__ U,
                                                     const cd* __restrict__ tws,
                                                     cd* __restrict__ scratch,
                                                     cd* __restrict__ oms) {
  const int b = blockIdx.x;
  if (!(req[b] & REQ_GRID)) return;
  const InstInfo in = info[b];
  const int K = Kev[b], M = in.nobs, N = in.N, P = in.P, logP = in.logP;
  const int64_t mo = in.obsoff;
  const int tid = threadIdx.x;
  extern __shared__ cd lds_sh[];
  __shared__ cd s_tw[FFT_TWL];
  __shared__ double red[SFO_NT / 64];
  load_tw_head<SFO_NT>(s_tw, tws);
  double p2[1] = {0.0};
  for (int m = tid; m < M; m += SFO_NT) p2[0] += phi ? cabs2(phi[mo + m]) : 1.0;
  block_sum<SFO_NT, 1>(p2, red);
  double* acc = reinterpret_cast<double*>(scratch + in.poff);  // P running sums
  const cd* Ub = U + in.uoff;
  auto body = [&](cd* __restrict__ buf) __attribute__((always_inline)) {
    for (int t = tid; t < P; t += SFO_NT) acc[t] = 0.0;
    for (int j = 0; j < K; ++j) {
      for (int t = tid; t < P; t += SFO_NT) buf[pidx(t)] = cd{0.0, 0.0};
      __syncthreads();
      for (int m = tid; m < M; m += SFO_NT) buf[pidx(idx[mo + m])] = Ub[(int64_t)j * M + m];
      __syncthreads();
      dif_fftn<SFO_NT>(buf, buf, 1, logP, false, false, s_tw, tws);
      for (int t = tid; t < P; t += SFO_NT) acc[t] += cabs2(buf[pidx(t)]);
      __syncthreads();
    }
    for (int t = tid; t < P; t += SFO_NT) buf[pidx(t)] = cd{acc[t], 0.0};
    __syncthreads();
    dit_fftn<SFO_NT>(buf, buf, 1, logP, true, true, s_tw, tws);
    const double ib = 1.0 / beta[b], sc = ib / (double)P;
    for (int t = tid; t < P; t += SFO_NT) {
      const bool lag = t < N || t > P - N;
      cd o{0.0, 0.0};
      if (lag) {
        const cd r = buf[pidx(t)];  // P sum_n sum_j U_nj conj(U_{n-t,j}), i.e. lag -t
        o = cd{-r.x * sc, r.y * sc};  // the lag +t sum is its conjugate
        if (t == 0) o.x += p2[0] * ib;
      }
      oms[in.poff + t] = o;
    }
    __syncthreads();
  };
  if (P > CONV_LDS_P) body(scratch + in.poff + 4 * (int64_t)P);
  else body(lds_sh);
}

// ---------------------------------------------------------------------------
// q and s at the grid candidates (FP64 direct sums over the observed samples).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(SF_NT) void k_sf_cand(const InstInfo* __restrict__ info,
                                                   const int32_t* __restrict__ req,
                                                   const int32_t* __restrict__ Kev,
                                                   const double* __restrict__ beta,
                                                   const int32_t* __restrict__ idx,
                                                   const cd* __restrict__ phi,
                                                   const cd* __restrict__ wM,
                                                   const cd* __restrict__ U,
                                                   const int32_t* __restrict__ cand,
                                                   const int32_t* __restrict__ ncand,
                                                   cd* __restrict__ cq, double* __restrict__ cs) {
  const int b = blockIdx.x / SF_CANDB, sub = blockIdx.x % SF_CANDB;
  if (!(req[b] & REQ_GRID)) return;
  const InstInfo in = info[b];
  const int K = Kev[b], M = in.nobs;
  const int64_t mo = in.obsoff;
  const int tid = threadIdx.x;
  const double ib = 1.0 / beta[b];
  const cd* Ub = U + in.uoff;
  const int B1 = SF_TB1(in.N), W = SF_TBW(in.N);
  __shared__ double red[34 * (SF_NT / 64)];
  extern __shared__ cd sf_lds[];  // the candidate's phase tables (W entries)
  const int nc = ncand[b];
  for (int c = sub; c < nc; c += SF_CANDB) {
    const double th = (double)cand[in.coff + c] / (double)in.L;
    __syncthreads();
    for (int j = tid; j < W; j += SF_NT)
      sf_lds[j] = cis2pi(frac_mul(j < B1 ? 64.0 * (double)j : (double)(j - B1), th));
    __syncthreads();
    double qa[3] = {0.0, 0.0, 0.0};  // q (re, im), sum |phi|^2
    for (int m = tid; m < M; m += SF_NT) {
      const cd ph = sf_phi(phi, mo + m);
      const cd t = cmulc(cmulc(wM[mo + m], ph), sf_cis(sf_lds, W, B1, 0, idx[mo + m]));
      qa[0] += t.x;
      qa[1] += t.y;
      qa[2] += cabs2(ph);
    }
    block_sum<SF_NT, 3>(qa, red);
    double sq = 0.0;  // sum_j |psi^H U_j|^2
    for (int j0 = 0; j0 < K; j0 += 16) {
      double acc[32];
#pragma unroll
      for (int q = 0; q < 32; ++q) acc[q] = 0.0;
      for (int m = tid; m < M; m += SF_NT) {
        const cd e = cconj(sf_cis(sf_lds, W, B1, 0, idx[mo + m]));
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
          if (j0 + jj >= K) break;
          const cd t = cmul(e, Ub[(int64_t)(j0 + jj) * M + m]);
          acc[2 * jj] += t.x;
          acc[2 * jj + 1] += t.y;
        }
      }
      block_sum<SF_NT, 32>(acc, red);
      for (int jj = 0; jj < 16 && j0 + jj < K; ++jj)
        sq = fma(acc[2 * jj], acc[2 * jj], fma(acc[2 * jj + 1], acc[2 * jj + 1], sq));
    }
    if (tid == 0) {
      cq[in.coff + c] = cd{qa[0], qa[1]};
      cs[in.coff + c] = (qa[2] - sq) * ib;
    }
  }
}

// ---------------------------------------------------------------------------
hipError_t launch_sf_eval(const InstInfo* info, const int32_t* req, const int32_t* Kev,
                          const double* theta, const double* gamma, const double* beta,
                          const void* y, int ydtype, const int32_t* idx, const cd* phi,
                          cd* sfm, cd* h, cd* cvec, cd* tabs, cd* wM, double* logdet, double* yCy,
                          double* ww, int32_t* status, cd* oq, cd* orr, cd* ou, cd* os, cd* ot,
                          cd* ov, cd* ox, int B, hipStream_t st) {
  hipLaunchKernelGGL(k_sf_tables, dim3(B), dim3(SF_NT), 0, st, info, req, Kev, theta, tabs);
  if (ydtype == 0) {
    (void)hipFuncSetAttribute((const void*)k_sf_gram<cf>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)SFG_LDS);
    hipLaunchKernelGGL(k_sf_gram<cf>, dim3(B), dim3(SFG_NT), SFG_LDS, st, info, req, Kev, tabs,
                       (const cf*)y, idx, phi, sfm, h);
  } else {
    (void)hipFuncSetAttribute((const void*)k_sf_gram<cd>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)SFG_LDS);
    hipLaunchKernelGGL(k_sf_gram<cd>, dim3(B), dim3(SFG_NT), SFG_LDS, st, info, req, Kev, tabs,
                       (const cd*)y, idx, phi, sfm, h);
  }
  const size_t shm = (size_t)2 * SF_KMAX * SF_LDK * sizeof(cd);
  (void)hipFuncSetAttribute((const void*)k_sf_solve, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)shm);
  hipLaunchKernelGGL(k_sf_solve, dim3(B), dim3(SF_NT), shm, st, info, req, Kev, gamma, beta, sfm,
                     h, cvec, os, ot, ov, ox, logdet, status);
  if (ydtype == 0)
    hipLaunchKernelGGL(k_sf_resid<cf>, dim3(B), dim3(SF_NT), 0, st, info, req, Kev, theta, beta,
                       (const cf*)y, idx, phi, tabs, cvec, status, wM, yCy, ww, oq, orr, ou);
  else
    hipLaunchKernelGGL(k_sf_resid<cd>, dim3(B), dim3(SF_NT), 0, st, info, req, Kev, theta, beta,
                       (const cd*)y, idx, phi, tabs, cvec, status, wM, yCy, ww, oq, orr, ou);
  return hipGetLastError();
}

hipError_t launch_sf_grid_inputs(const InstInfo* info, const int32_t* req, const int32_t* Kev,
                                 const double* theta, const double* gamma, const double* beta,
                                 const int32_t* idx, const cd* phi, const cd* wM, const cd* sfm,
                                 const cd* tabs, const cd* tws, cd* w, cd* U, cd* scratch,
                                 cd* oms, int B, int maxP, hipStream_t st) {
  const size_t shp = (size_t)(SF_UMT + SF_KMAX) * SF_LDK * sizeof(cd);
  (void)hipFuncSetAttribute((const void*)k_sf_prep, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)shp);
  hipLaunchKernelGGL(k_sf_prep, dim3(B), dim3(SF_NT), shp, st, info, req, Kev, theta, gamma, idx,
                     phi, wM, sfm, tabs, w, U);
  const size_t sho = (size_t)padded(maxP < CONV_LDS_P ? maxP : CONV_LDS_P) * sizeof(cd);
  (void)hipFuncSetAttribute((const void*)k_sf_omega, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)sho);
  hipLaunchKernelGGL(k_sf_omega, dim3(B), dim3(SFO_NT), sho, st, info, req, Kev, beta, idx, phi,
                     U, tws, scratch, oms);
  return hipGetLastError();
}

hipError_t launch_sf_cand(const InstInfo* info, const int32_t* req, const int32_t* Kev,
                          const double* beta, const int32_t* idx, const cd* phi, const cd* wM,
                          const cd* U, const int32_t* cand, const int32_t* ncand, cd* cq, double* cs,
                          int B, int maxN, hipStream_t st) {
  const size_t shc = (size_t)SF_TBW(maxN) * sizeof(cd);
  (void)hipFuncSetAttribute((const void*)k_sf_cand, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)shc);
  hipLaunchKernelGGL(k_sf_cand, dim3(B * SF_CANDB), dim3(SF_NT), shc, st, info, req, Kev, beta,
                     idx, phi, wM, U, cand, ncand, cq, cs);
  return hipGetLastError();
}

}  // namespace sfls

namespace sfls {

// Validation of the observation arrays before any kernel uses them as
// indices: instance b's indices must be strictly increasing in [0, N) and its
// weights (when given) nonzero and finite; bad[b] = 1 otherwise.
__global__ __launch_bounds__(SF_NT) void k_sf_check(const InstInfo* __restrict__ info,
                                                    const int32_t* __restrict__ idx,
                                                    const cd* __restrict__ phi,
                                                    int32_t* __restrict__ bad) {
  const int b = blockIdx.x;
  const InstInfo in = info[b];
  const int64_t mo = in.obsoff;
  int err = 0;
  for (int m = threadIdx.x; m < in.nobs; m += SF_NT) {
    const int32_t n = idx[mo + m];
    if (n < 0 || n >= in.N) err = 1;
    if (m > 0 && !(idx[mo + m - 1] < n)) err = 1;
    if (phi) {
      const cd p = phi[mo + m];
      const double a = cabs2(p);
      if (!(a > 0.0) || !isfinite(a)) err = 1;
    }
  }
  err = __syncthreads_or(err);
  if (threadIdx.x == 0) bad[b] = err;
}

hipError_t launch_sf_check(const InstInfo* info, const int32_t* idx, const cd* phi, int32_t* bad,
                           int B, hipStream_t st) {
  hipLaunchKernelGGL(k_sf_check, dim3(B), dim3(SF_NT), 0, st, info, idx, phi, bad);
  return hipGetLastError();
}

}  // namespace sfls
