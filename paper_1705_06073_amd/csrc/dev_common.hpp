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
// In-LDS radix-2 FFT of n = 2^logn points with NT threads.
//   dif_fft: natural order in -> bit-reversed order out, kernel exp(sgn j 2pi kn/n)
//   dit_fft: bit-reversed in -> natural order out, kernel exp(sgn j 2pi kn/n)
// Twiddles come from the stage-major table tws[h + pos] = exp(-j 2 pi pos / 2h)
// (h a power of two, pos < h), so the twiddles of one stage are contiguous.
// No scaling.  Both end with a barrier.
// ---------------------------------------------------------------------------
template <typename C, int NT>
__device__ void dif_fft(C* x, int logn, int sgn, const C* __restrict__ tws) {
  const int n = 1 << logn;
  for (int lh = logn - 1; lh >= 0; --lh) {
    const int h = 1 << lh;
    for (int b = threadIdx.x; b < (n >> 1); b += NT) {
      const int pos = b & (h - 1);
      const int i = ((b >> lh) << (lh + 1)) + pos;
      const int j = i + h;
      C u = x[i], v = x[j];
      C w = tws[h + pos];
      if (sgn > 0) w.y = -w.y;
      x[i] = cadd(u, v);
      x[j] = cmul(csub(u, v), w);
    }
    __syncthreads();
  }
}

template <typename C, int NT>
__device__ void dit_fft(C* x, int logn, int sgn, const C* __restrict__ tws) {
  const int n = 1 << logn;
  for (int lh = 0; lh < logn; ++lh) {
    const int h = 1 << lh;
    for (int b = threadIdx.x; b < (n >> 1); b += NT) {
      const int pos = b & (h - 1);
      const int i = ((b >> lh) << (lh + 1)) + pos;
      const int j = i + h;
      C w = tws[h + pos];
      if (sgn > 0) w.y = -w.y;
      C u = x[i], v = cmul(x[j], w);
      x[i] = cadd(u, v);
      x[j] = csub(u, v);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ int bitrev(int v, int logn) {
  return (int)(__brev((unsigned)v) >> (32 - logn));
}

}  // namespace sfls
