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
  int64_t poff;   // P-length scratch
  int64_t goff;   // L-length grid arrays
  int64_t koff;   // component arrays
  int64_t ooff;   // 2N-1 omega arrays (sfls_omega)
  int64_t coff;   // candidate arrays
};

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
constexpr int SCH_DIRECT = 128;

// Per-instance layout of the recursion's scratch (offsets in complex elements).
struct SchurLayout {
  int64_t scr_off;
  int64_t act_off;
  int32_t nact;
  int32_t Fmax;
  int64_t win[SCH_MAXL];   // right-child windows (u then v, mmax[l] each)
  int64_t res[SCH_MAXL];   // Theta results, 2 sides x 4 polynomials x mmax[l]
  int64_t spec[SCH_MAXL];  // Theta1 spectra, 4 x F
  int32_t mmax[SCH_MAXL];
};

}  // namespace sfls
