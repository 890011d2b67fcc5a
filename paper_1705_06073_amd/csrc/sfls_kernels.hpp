// Kernel-side data structures and launch wrappers of the superfast-LSE path.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dev_common.hpp"

namespace sfls {

// Per-instance sizes and offsets, prepared on the host for every call.
struct InstInfo {
  int32_t N;      // samples
  int32_t P;      // convolution FFT size, power of two >= 2N-1
  int32_t logP;
  int32_t M;      // grid sub-FFT size, power of two >= N
  int32_t logM;
  int32_t R;      // L / M residues
  int32_t L;      // grid size
  int32_t kcap;   // component capacity
  int64_t off;    // per-sample arrays (y, c, rho, delta, w)
  int64_t poff;   // scratch: 4 blocks of P, then (P > CONV_LDS_P) a transform buffer
  int64_t goff;   // L-length grid arrays
  int64_t koff;   // component arrays
  int64_t ooff;   // 2N-1 omega arrays (sfls_omega)
  int64_t coff;   // candidate arrays
  // incomplete observations (Sec. IV): the instance observes nobs samples,
  // its observation arrays (y, indices, weights, C^{-1} y) start at obsoff;
  // nobs = 0 for complete data (y of N samples at off)
  int32_t nobs;
  int32_t pad_;
  int64_t obsoff;
  int64_t sfoff;  // semifast K x K matrices (4 kcap^2 complex elements)
  int64_t uoff;   // semifast grid columns (nobs x kcap complex elements)
  int64_t tboff;  // semifast phase tables (kcap x (ceil(N/64) + 64) complex elements)
};

// Semifast phase tables: e^{j 2 pi n theta_k} = T1_k[n >> 6] T2_k[n & 63] with
// T1_k[a] = e^{j 2 pi 64 a theta_k}, T2_k[b] = e^{j 2 pi b theta_k}, each entry
// from an exactly reduced phase; a component's tables are SF_TB1(N) + 64 entries.
__host__ __device__ constexpr int SF_TB1(int N) { return (N + 63) / 64; }
__host__ __device__ constexpr int SF_TBW(int N) { return SF_TB1(N) + 64; }

// Observation vectors of a launch (the multiple-measurement-vector model of
// Sec. V; G = 1 is the single-vector model).  Every instance of a launch has
// G vectors that share its generator: vector g of instance b is the signal at
// y + g ystride + off, its C^{-1} y at w + g wstride + off, its active-set
// vectors q, r, u at ev + g kstride + koff, its candidates' q at
// cq + g cstride + coff.
struct Vecs {
  int32_t G = 1;
  int64_t ystride = 0, wstride = 0, kstride = 0, cstride = 0;
};

// Largest P whose transform buffer sits in LDS (P = 8192 fills one CU's LDS
// with the twiddle head); larger transforms run the same passes on a buffer of
// padded(P) in the instance's scratch, after its four P blocks.
constexpr int CONV_LDS_P = 8192;
// Largest grid sub-FFT size M (two buffers of padded(M) in LDS): M = min(2^ceil(log2 N), cap).
constexpr int GRID_LOGM_F32 = 13;
constexpr int GRID_LOGM_F64 = 12;

// Active vectors by NUFFT (Gaussian gridding): half-width of the spreading
// window in grid points (2 NU_MSP points per frequency; relative error below
// 1e-14 at an oversampling of at least 2), and the work (points x N) from
// which the automatic choice prefers it to the direct sums.
constexpr int NU_MSP = 16;
constexpr double NU_MIN_WORK = 8388608.0;
// The covariance column (a1) by the type-1 NUFFT: at most this many
// frequencies (their sort keys stay in LDS), only where the P-point transform
// lives in the instance's scratch (P > CONV_LDS_P), and in the automatic mode
// from K N >= NUC_MIN_WORK.
constexpr int NUC_KMAX = 2048;
constexpr double NUC_MIN_WORK = 2097152.0;
__host__ __device__ inline bool use_nufft_col(int mode, int N, int P, int K) {
  if (mode == 1 || K <= 0 || K > NUC_KMAX || P <= CONV_LDS_P) return false;
  if (mode == 2) return true;
  return (double)K * (double)N >= NUC_MIN_WORK;
}

// Incomplete observations (Sec. IV): largest number of active components of
// the semifast evaluation (its K x K factor and inverse stay in LDS).
constexpr int SF_KMAX = 64;

// Request bits of one instance for the current evaluation round.
enum : int32_t { REQ_EVAL = 1, REQ_GRID = 2, REQ_APPROX = 4 };

// Coefficients of the separable forms of s, t, v, x: for each quantity a 4x4
// matrix C[a][b] with  Q = delta^{-1} sum_ab C[a][b] G_a conj(G_b),
// G_a(theta) = sum_q (q-c)^a rho_q e^{-j 2 pi q theta}, c = (N-1)/2.
struct SepCoef {
  double c[4][16];  // s, t, v, x
};

// Superfast Schur: one action of the flattened recursion.
enum : int32_t { SCH_LEAF_ACT = 0, SCH_MID = 1, SCH_POST = 2, SCH_ROOT = 3, SCH_ROOT_LEAF = 4 };
struct SchurAct {
  int32_t type, n0, m, m1, level, side, win_level, logF;
};
constexpr int SCH_MAXL = 16;
// Merges of windows up to this size use direct polynomial products (parallel
// sums, no transforms; the transform buffers must then hold 8m + 256 elements
// each); larger ones use FFTs of size >= m.
constexpr int SCH_DIRECT = 64;
// Transform merges with F above this use two buffers of padded(F) in the
// instance's Schur scratch (at xbig) instead of LDS (default; a context can
// lower it, down to SCH_LDS_F_MIN, so that more instances share a CU's LDS).
constexpr int SCH_LDS_F = 4096;
constexpr int SCH_LDS_F_MIN = 256;

// Per-instance layout of the recursion's scratch (offsets in complex elements).
struct SchurLayout {
  int64_t scr_off;
  int64_t act_off;
  int32_t nact;
  int32_t Fmax;
  int32_t ldsF;            // transform merges with F > ldsF run on scratch (at xbig)
  int32_t pad_;
  int64_t win[SCH_MAXL];   // right-child windows (u then v, mmax[l] each)
  int64_t res[SCH_MAXL];   // Theta results, 2 sides x 4 polynomials x mmax[l]
  int64_t spec[SCH_MAXL];  // Theta1 first-row spectra, 2 x F
  int64_t xbig;            // transform buffers of merges with F > SCH_LDS_F
  int32_t mmax[SCH_MAXL];
};

// Outputs of one finished instance, packed by k_gather_results for a single
// device-to-host copy (components follow in a separate packed array).
// One admission: the slot whose tables k_admit copies from pinned host
// memory, and the signal to copy into the pool (src NULL: already there).
struct AdmitRec {
  int32_t slot;
  int32_t pad_;
  const void* src;
  int64_t dst_bytes;  // byte offset in the signal pool
  int64_t bytes;
};

struct SlotResult {
  int64_t K;
  double beta, zeta, obj;
  int32_t iters, evals, status, slot;
};

}  // namespace sfls
