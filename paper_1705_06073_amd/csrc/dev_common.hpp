// Device helpers shared by the gfx950 kernels: complex arithmetic, exact
// phase reduction, wave64 reductions through DPP, and an in-LDS radix-2 FFT.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sfls {

struct cd { double x, y; };
struct cf { float x, y; };

template <typename R> struct cpx;
template <> struct cpx<double> { using T = cd; };
template <> struct cpx<float> { using T = cf; };

template <typename C> __device__ __forceinline__ C mk(decltype(C{}.x) a, decltype(C{}.x) b) { return C{a, b}; }

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return C{fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x)};
}
// a * conj(b)
template <typename C> __device__ __forceinline__ C cmulc(C a, C b) {
  return C{fma(a.x, b.x, a.y * b.y), fma(a.y, b.x, -a.x * b.y)};
}
// acc + a * b
template <typename C> __device__ __forceinline__ C cfma(C a, C b, C acc) {
  return C{fma(a.x, b.x, fma(-a.y, b.y, acc.x)), fma(a.x, b.y, fma(a.y, b.x, acc.y))};
}
// acc + a * conj(b)
template <typename C> __device__ __forceinline__ C cfmac(C a, C b, C acc) {
  return C{fma(a.x, b.x, fma(a.y, b.y, acc.x)), fma(a.y, b.x, fma(-a.x, b.y, acc.y))};
}
template <typename C> __device__ __forceinline__ C cconj(C a) { return C{a.x, -a.y}; }
template <typename C, typename R> __device__ __forceinline__ C cscale(C a, R s) { return C{a.x * s, a.y * s}; }
template <typename C> __device__ __forceinline__ auto cabs2(C a) { return fma(a.x, a.x, a.y * a.y); }

__device__ __forceinline__ cf to_f(cd a) { return cf{(float)a.x, (float)a.y}; }
__device__ __forceinline__ cd to_d(cf a) { return cd{(double)a.x, (double)a.y}; }

// (n * th) mod 1 in [-1/2, 1/2] with the product error recovered by an FMA,
// so the phase stays accurate to ~1 ulp of 1/2 for |n| < 2^30.  Contraction
// must stay off here: fusing p - rint(p) into fma(n, th, -rint(p)) would
// count the rounding error of p twice.
__device__ __forceinline__ double frac_mul(double n, double th) {
#pragma clang fp contract(off)
  double p = n * th;
  double e = fma(n, th, -p);
  double r = p - rint(p);
  return r + e;
}

// exp(j 2 pi f), f a reduced fraction.
__device__ __forceinline__ cd cis2pi(double f) {
  double s, c;
  sincospi(2.0 * f, &s, &c);
  return cd{c, s};
}

// exp(j 2 pi k / m) for integers with 0 <= k < m, m a power of two, evaluated
// from the exact fraction k/m.
__device__ __forceinline__ cd cis_frac(int64_t k, int64_t m) {
  double f = (double)k / (double)m;  // exact for m = 2^e <= 2^53
  if (f > 0.5) f -= 1.0;
  return cis2pi(f);
}

// ---------------------------------------------------------------------------
// wave64 reductions.  The xor-butterfly gives bitwise-identical sums in every
// lane (each pairwise add is commutative), so all lanes can branch on them.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
  int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// sum over the 64 lanes, identical in every lane
__device__ __forceinline__ double wave_sum(double v) {
  v = v + dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v = v + dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v = v + dpp_f64<0x141>(v);  // row_half_mirror
  v = v + dpp_f64<0x140>(v);  // row_mirror
  double r0 = readlane_f64(v, 0), r1 = readlane_f64(v, 16);
  double r2 = readlane_f64(v, 32), r3 = readlane_f64(v, 48);
  return (r0 + r1) + (r2 + r3);
}

__device__ __forceinline__ float wave_sum_f(float v) {
  v = v + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
  v = v + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false));
  v = v + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x141, 0xF, 0xF, false));
  v = v + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x140, 0xF, 0xF, false));
  float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
  float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
  float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
  float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
  return (r0 + r1) + (r2 + r3);
}

__device__ __forceinline__ cd wave_sum(cd v) { return cd{wave_sum(v.x), wave_sum(v.y)}; }

// Block-wide sum of NV doubles per thread for a block of NT threads; every
// thread receives the totals (summed over waves in a fixed order).
// `scratch` holds NV * (NT/64) doubles of LDS.
template <int NT, int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* scratch) {
  constexpr int W = NT / 64;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  if (W == 1) return;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) scratch[i * W + wv] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) s += scratch[i * W + w];
    v[i] = s;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// In-LDS FFT of n = 2^logn points with NT threads: the stages of a radix-2
// network, with up to 4 consecutive stages fused per LDS pass (a group holds
// 2^KS elements at stride s in registers).
//   dif: natural order in -> bit-reversed order out
//   dit: bit-reversed in -> natural order out
// Kernel exp(-j 2pi kn/n), or exp(+j 2pi kn/n) when conj is set.  Twiddle
// W_{2h}^pos = tws[h + pos] (stage-major table, h a power of two, pos < h).
// No scaling.  Buffers use the padded layout pidx (one pad slot after every
// 16 elements) so that strided and unit-stride passes spread over all banks.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int pidx(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int padded(int n) { return n + (n >> 4) + 1; }
// Twiddles of stages with 2h <= FFT_TWL may come from an LDS copy of the
// table head (FFT_TWL entries).
constexpr int FFT_TWL = 1024;

template <int KS, typename C>
__device__ __forceinline__ void dif_group(C* z, int g, int lh_top, const C* __restrict__ tws,
                                          bool conj) {
  constexpr int R = 1 << KS;
  const int ls = lh_top - KS + 1;
  const int s = 1 << ls;
  const int gl = g & (s - 1);
  const int base = gl + ((g >> ls) << (ls + KS));
  C x[R];
#pragma unroll
  for (int j = 0; j < R; ++j) x[j] = z[pidx(base + j * s)];
#pragma unroll
  for (int t = 0; t < KS; ++t) {
    const int hj = R >> (t + 1);
    const int h = hj << ls;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      if (j & hj) continue;
      C w = tws[h + gl + (j & (hj - 1)) * s];
      if (conj) w.y = -w.y;
      const C u = x[j], v = x[j + hj];
      x[j] = cadd(u, v);
      x[j + hj] = cmul(csub(u, v), w);
    }
  }
#pragma unroll
  for (int j = 0; j < R; ++j) z[pidx(base + j * s)] = x[j];
}

template <int KS, typename C>
__device__ __forceinline__ void dit_group(C* z, int g, int lh_bot, const C* __restrict__ tws,
                                          bool conj) {
  constexpr int R = 1 << KS;
  const int ls = lh_bot;
  const int s = 1 << ls;
  const int gl = g & (s - 1);
  const int base = gl + ((g >> ls) << (ls + KS));
  C x[R];
#pragma unroll
  for (int j = 0; j < R; ++j) x[j] = z[pidx(base + j * s)];
#pragma unroll
  for (int t = 0; t < KS; ++t) {
    const int hj = 1 << t;
    const int h = hj << ls;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      if (j & hj) continue;
      C w = tws[h + gl + (j & (hj - 1)) * s];
      if (conj) w.y = -w.y;
      const C u = x[j], v = cmul(x[j + hj], w);
      x[j] = cadd(u, v);
      x[j + hj] = csub(u, v);
    }
  }
#pragma unroll
  for (int j = 0; j < R; ++j) z[pidx(base + j * s)] = x[j];
}

// Largest number of stages per pass for na transforms of size 2^logn: small
// transforms use shorter groups so that more threads share a pass.
__device__ __forceinline__ int fft_ks_max(int na, int logn) {
  const int tot = na << logn;
  return tot >= 2048 ? 4 : (tot >= 512 ? 3 : 2);
}

// na (1 or 2) transforms of size 2^logn over the buffers x, y (conjugate
// kernels per buffer: cx, cy); ends with a barrier.  Twiddles of the passes
// whose stages all have 2h <= FFT_TWL come from tl (an LDS copy of the table
// head, or the global table itself), the others from the global table tg;
// those are always 4-stage passes (first DIF / last DIT pass of n > FFT_TWL).
// stop > 0 leaves the last `stop` stages (h < 2^stop) to the caller.
template <int NT, typename C>
__device__ __forceinline__ void dif_fftn(C* x, C* y, int na, int logn, bool cx, bool cy,
                                         const C* __restrict__ tl, const C* __restrict__ tg,
                                         int stop = 0) {
  const int km = fft_ks_max(na, logn);
  int lh = logn - 1;
  while (lh >= stop) {
    const int ks = lh + 1 - stop < km ? lh + 1 - stop : km;
    const int lg = logn - ks;  // log2(groups per transform)
    const int tot = na << lg;
    const bool lds_tw = (2 << lh) <= FFT_TWL;
    for (int gi = threadIdx.x; gi < tot; gi += NT) {
      const bool second = (gi >> lg) != 0;
      C* z = second ? y : x;
      const bool cj = second ? cy : cx;
      const int g = gi & ((1 << lg) - 1);
      if (!lds_tw) {
        dif_group<4>(z, g, lh, tg, cj);
        continue;
      }
      switch (ks) {
        case 4: dif_group<4>(z, g, lh, tl, cj); break;
        case 3: dif_group<3>(z, g, lh, tl, cj); break;
        case 2: dif_group<2>(z, g, lh, tl, cj); break;
        default: dif_group<1>(z, g, lh, tl, cj); break;
      }
    }
    __syncthreads();
    lh -= ks;
  }
}

// start > 0: the first `start` stages (h < 2^start) were done by the caller.
template <int NT, typename C>
__device__ __forceinline__ void dit_fftn(C* x, C* y, int na, int logn, bool cx, bool cy,
                                         const C* __restrict__ tl, const C* __restrict__ tg,
                                         int start = 0) {
  const int km = fft_ks_max(na, logn);
  const int rem = (logn - start) % km;
  int lb = start;
  while (lb < logn) {
    // the shorter pass first, so that the last (largest-h) pass has km stages
    const int ks = (lb == start && rem) ? rem : km;
    const int lg = logn - ks;
    const int tot = na << lg;
    const bool lds_tw = (2 << (lb + ks - 1)) <= FFT_TWL;
    for (int gi = threadIdx.x; gi < tot; gi += NT) {
      const bool second = (gi >> lg) != 0;
      C* z = second ? y : x;
      const bool cj = second ? cy : cx;
      const int g = gi & ((1 << lg) - 1);
      if (!lds_tw) {
        dit_group<4>(z, g, lb, tg, cj);
        continue;
      }
      switch (ks) {
        case 4: dit_group<4>(z, g, lb, tl, cj); break;
        case 3: dit_group<3>(z, g, lb, tl, cj); break;
        case 2: dit_group<2>(z, g, lb, tl, cj); break;
        default: dit_group<1>(z, g, lb, tl, cj); break;
      }
    }
    __syncthreads();
    lb += ks;
  }
}

// One wave's transform of size 2^logn in its own LDS buffer (padded layout,
// same kernels and orders as above).  The lanes exchange data through LDS
// between passes without a workgroup barrier: a wave's LDS accesses are
// performed in program order, and wave_sync keeps the compiler from moving
// accesses across a pass boundary.  Groups are sized so that the 64 lanes
// share each pass.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ __forceinline__ int wave_ks_max(int logn) {
  return logn >= 10 ? 4 : (logn == 9 ? 3 : 2);
}
// The passes of a size known at compile time, unrolled: the runtime loop
// over passes (with the group size chosen per pass) costs about as much as
// the pass itself at the sizes the one-wave transforms run.
template <int LOGN, int LH, typename C>
__device__ __forceinline__ void wave_dif_passes(C* z, bool cj, const C* __restrict__ tl,
                                                const C* __restrict__ tg, int lane) {
  if constexpr (LH >= 0) {
    constexpr int KM = LOGN >= 10 ? 4 : (LOGN == 9 ? 3 : 2);
    constexpr int KS = LH + 1 < KM ? LH + 1 : KM;
    constexpr int TOT = 1 << (LOGN - KS);
    constexpr bool LDS_TW = (2 << LH) <= FFT_TWL;
#pragma unroll
    for (int g0 = 0; g0 < TOT; g0 += 64) {
      const int g = g0 + lane;
      if (TOT < 64 && g >= TOT) continue;
      if constexpr (LDS_TW) dif_group<KS>(z, g, LH, tl, cj);
      else dif_group<4>(z, g, LH, tg, cj);
    }
    wave_sync();
    wave_dif_passes<LOGN, LH - KS>(z, cj, tl, tg, lane);
  }
}
template <int LOGN, int LB, typename C>
__device__ __forceinline__ void wave_dit_passes(C* z, bool cj, const C* __restrict__ tl,
                                                const C* __restrict__ tg, int lane) {
  if constexpr (LB < LOGN) {
    constexpr int KM = LOGN >= 10 ? 4 : (LOGN == 9 ? 3 : 2);
    constexpr int REM = LOGN % KM;
    constexpr int KS = (LB == 0 && REM) ? REM : KM;
    constexpr int TOT = 1 << (LOGN - KS);
    constexpr bool LDS_TW = (2 << (LB + KS - 1)) <= FFT_TWL;
#pragma unroll
    for (int g0 = 0; g0 < TOT; g0 += 64) {
      const int g = g0 + lane;
      if (TOT < 64 && g >= TOT) continue;
      if constexpr (LDS_TW) dit_group<KS>(z, g, LB, tl, cj);
      else dit_group<4>(z, g, LB, tg, cj);
    }
    wave_sync();
    wave_dit_passes<LOGN, LB + KS>(z, cj, tl, tg, lane);
  }
}
template <typename C>
__device__ __forceinline__ void wave_dif(C* z, int logn, bool cj, const C* __restrict__ tl,
                                         const C* __restrict__ tg, int lane) {
  switch (logn) {
    case 7: wave_dif_passes<7, 6>(z, cj, tl, tg, lane); return;
    case 8: wave_dif_passes<8, 7>(z, cj, tl, tg, lane); return;
    case 9: wave_dif_passes<9, 8>(z, cj, tl, tg, lane); return;
    case 10: wave_dif_passes<10, 9>(z, cj, tl, tg, lane); return;
    default: break;
  }
  const int km = wave_ks_max(logn);
  int lh = logn - 1;
  while (lh >= 0) {
    const int ks = lh + 1 < km ? lh + 1 : km;
    const int tot = 1 << (logn - ks);
    const bool lds_tw = (2 << lh) <= FFT_TWL;
    for (int g = lane; g < tot; g += 64) {
      if (!lds_tw) {
        dif_group<4>(z, g, lh, tg, cj);
        continue;
      }
      switch (ks) {
        case 4: dif_group<4>(z, g, lh, tl, cj); break;
        case 3: dif_group<3>(z, g, lh, tl, cj); break;
        case 2: dif_group<2>(z, g, lh, tl, cj); break;
        default: dif_group<1>(z, g, lh, tl, cj); break;
      }
    }
    wave_sync();
    lh -= ks;
  }
}
template <typename C>
__device__ __forceinline__ void wave_dit(C* z, int logn, bool cj, const C* __restrict__ tl,
                                         const C* __restrict__ tg, int lane) {
  switch (logn) {
    case 7: wave_dit_passes<7, 0>(z, cj, tl, tg, lane); return;
    case 8: wave_dit_passes<8, 0>(z, cj, tl, tg, lane); return;
    case 9: wave_dit_passes<9, 0>(z, cj, tl, tg, lane); return;
    case 10: wave_dit_passes<10, 0>(z, cj, tl, tg, lane); return;
    default: break;
  }
  const int km = wave_ks_max(logn);
  const int rem = logn % km;
  int lb = 0;
  while (lb < logn) {
    const int ks = (lb == 0 && rem) ? rem : km;
    const int tot = 1 << (logn - ks);
    const bool lds_tw = (2 << (lb + ks - 1)) <= FFT_TWL;
    for (int g = lane; g < tot; g += 64) {
      if (!lds_tw) {
        dit_group<4>(z, g, lb, tg, cj);
        continue;
      }
      switch (ks) {
        case 4: dit_group<4>(z, g, lb, tl, cj); break;
        case 3: dit_group<3>(z, g, lb, tl, cj); break;
        case 2: dit_group<2>(z, g, lb, tl, cj); break;
        default: dit_group<1>(z, g, lb, tl, cj); break;
      }
    }
    wave_sync();
    lb += ks;
  }
}

// small bundles of complex values loaded together
struct cd2 { cd a, b; };
struct cd3 { cd a, b, c; };
struct cd4 { cd a, b, c, d; };

// for (t = first; t < n; t += step) use(t, ld(t)), with the loads of U
// consecutive iterations issued before any of their uses: a loop that stages
// global data into LDS otherwise waits for each load in turn.
template <int U, typename Ld, typename Use>
__device__ __forceinline__ void batched_for(int first, int step, int n, Ld ld, Use use) {
  using V = decltype(ld(0));
  for (int t0 = first; t0 < n; t0 += U * step) {
    V v[U];
#pragma unroll
    for (int i = 0; i < U; ++i) {
      const int t = t0 + i * step;
      if (t < n) v[i] = ld(t);
    }
#pragma unroll
    for (int i = 0; i < U; ++i) {
      const int t = t0 + i * step;
      if (t < n) use(t, v[i]);
    }
  }
}

// Copy the head of the stage-major twiddle table to LDS (caller syncs).
template <int NT, typename C>
__device__ __forceinline__ void load_tw_head(C* tl, const C* __restrict__ tg) {
  for (int t = threadIdx.x; t < FFT_TWL; t += NT) tl[t] = tg[t];
}

__device__ __forceinline__ int bitrev(int v, int logn) {
  return (int)(__brev((unsigned)v) >> (32 - logn));
}

}  // namespace sfls
