// a9 on the device: one wave per instance runs the estimator's state machine
// between evaluation rounds; plus small setup kernels.
#include "k_launch.hpp"

namespace sfls {

// One wave as the driver's team.  The folds combine lanes in an xor-butterfly
// (every step pairs the same two operands in either order) and finish in
// scalar registers, so every lane holds the same bits.
template <typename Op>
__device__ __forceinline__ double wave_fold(double v, Op op) {
  v = op(v, dpp_f64<0xB1>(v));   // quad_perm [1,0,3,2]
  v = op(v, dpp_f64<0x4E>(v));   // quad_perm [2,3,0,1]
  v = op(v, dpp_f64<0x141>(v));  // row_half_mirror
  v = op(v, dpp_f64<0x140>(v));  // row_mirror
  const double r0 = readlane_f64(v, 0), r1 = readlane_f64(v, 16);
  const double r2 = readlane_f64(v, 32), r3 = readlane_f64(v, 48);
  return op(op(r0, r1), op(r2, r3));
}
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}
struct WaveTeam {
  __device__ static int lane() { return threadIdx.x & 63; }
  __device__ static int width() { return 64; }
  __device__ static double sum(double v) { return wave_sum(v); }
  __device__ static double max(double v) {
    return wave_fold(v, [](double a, double b) { return fmax(a, b); });
  }
  __device__ static double min(double v) {
    return wave_fold(v, [](double a, double b) { return fmin(a, b); });
  }
  __device__ static int imin(int v) {
    v = ::min(v, dpp_i32<0xB1>(v));
    v = ::min(v, dpp_i32<0x4E>(v));
    v = ::min(v, dpp_i32<0x141>(v));
    v = ::min(v, dpp_i32<0x140>(v));
    const int r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
    const int r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
    return ::min(::min(r0, r1), ::min(r2, r3));
  }
  __device__ static bool any(bool b) { return __ballot(b) != 0; }
  // lanes exchange data through memory: keep the compiler from reordering
  // accesses across this point (a wave's accesses reach memory in order)
  __device__ static void sync() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }
};

__global__ __launch_bounds__(64) void k_driver(const InstInfo* __restrict__ info,
                                               const DrvParams* __restrict__ prm, DrvPools p,
                                               int B, int pass) {
  const int b = blockIdx.x;
  if (b >= B) return;
  if (pass == 1 && !(p.req2 && p.req2[b] != 0)) return;
  if (pass == 0 && p.req2) {
    // a request with a grid sweep waits for the round's grid stage, which
    // runs after this pass (its evaluation, if any, is done); pass 1 steps it
    const int32_t r0 = p.req[b];
    if (r0 & REQ_GRID) {
      if (threadIdx.x == 0) p.req2[b] = r0 & ~REQ_EVAL;
      return;
    }
  }
  const InstInfo in = info[b];
  DrvState S = p.st[b];
  if (S.phase == PH_DONE) return;
  if (pass == 2 && S.phase != PH_START) return;
  const int64_t ko = in.koff, k2 = 2 * in.koff, co = in.coff;
  const int J = prm->J;
  DrvArrays A;
  A.N = in.N;
  A.Mo = in.nobs > 0 ? in.nobs : in.N;
  A.L = in.L;
  A.kcap = in.kcap;
  A.G = p.G;
  A.vk = 2 * p.kstride;
  A.vc = 2 * p.cstride;
  A.vo = 2 * p.ostride;
  A.th = p.th + ko;
  A.ga = p.ga + ko;
  A.th_e = p.th_e + ko;
  A.ga_e = p.ga_e + ko;
  A.K_e = p.K_e + b;
  A.beta_e = p.beta_e + b;
  A.req = p.req + b;
  A.gbar_e = p.gbar_e + b;
  A.zeta_e = p.zeta_e + b;
  A.g = p.g + k2;
  A.d = p.d + k2;
  A.gt = p.gt + k2;
  A.q_save = p.q_save + k2;
  A.Sm = p.Sm + (int64_t)J * k2;
  A.Ym = p.Ym + (int64_t)J * k2;
  A.rhom = p.rhom + (int64_t)J * b;
  A.am = p.am + (int64_t)J * b;
  A.ev_q = reinterpret_cast<double*>(p.ev_q + ko);
  A.ev_r = reinterpret_cast<double*>(p.ev_r + ko);
  A.ev_u = reinterpret_cast<double*>(p.ev_u + ko);
  A.ev_s = reinterpret_cast<double*>(p.ev_s + ko);
  A.ev_t = reinterpret_cast<double*>(p.ev_t + ko);
  A.ev_v = reinterpret_cast<double*>(p.ev_v + ko);
  A.ev_x = reinterpret_cast<double*>(p.ev_x + ko);
  A.logdet = p.logdet + b;
  A.yCy = p.yCy + b;
  A.ww = p.ww + b;
  A.lev_status = p.lev_status + b;
  A.cand = p.cand + co;
  A.ncand = p.ncand + b;
  A.cand_q = reinterpret_cast<const double*>(p.cand_q + co);
  A.cand_s = p.cand_s + co;
  A.cbuf_dl = p.cbuf_dl + co;
  A.cbuf_gh = p.cbuf_gh + co;
  A.cbuf_l = p.cbuf_l + co;
  const int64_t oo = p.out_koff[b];
  A.out_K = p.out_K + b;
  A.out_theta = p.out_theta + oo;
  A.out_alpha = reinterpret_cast<double*>(p.out_alpha + oo);
  A.out_gamma = p.out_gamma + oo;
  A.out_beta = p.out_beta + b;
  A.out_zeta = p.out_zeta + b;
  A.out_obj = p.out_obj + b;
  A.out_iters = p.out_iters + b;
  A.out_evals = p.out_evals ? p.out_evals + b : nullptr;
  A.out_status = p.out_status + b;
  if (p.nsh > 0) {
    const int bs = b + p.nsh;
    const int64_t ks = info[bs].koff;
    A.sh_th_e = p.th_e + ks;
    A.sh_ga_e = p.ga_e + ks;
    A.sh_K_e = p.K_e + bs;
    A.sh_beta_e = p.beta_e + bs;
    A.sh_gbar_e = p.gbar_e + bs;
    A.sh_zeta_e = p.zeta_e + bs;
    A.sh_req = p.req + bs;
    A.sh_wish = p.wish + b;
    A.sh_ev_q = reinterpret_cast<const double*>(p.ev_q + ks);
    A.sh_ev_r = reinterpret_cast<const double*>(p.ev_r + ks);
    A.sh_ev_u = reinterpret_cast<const double*>(p.ev_u + ks);
    A.sh_ev_s = reinterpret_cast<const double*>(p.ev_s + ks);
    A.sh_ev_t = reinterpret_cast<const double*>(p.ev_t + ks);
    A.sh_ev_v = reinterpret_cast<const double*>(p.ev_v + ks);
    A.sh_ev_x = reinterpret_cast<const double*>(p.ev_x + ks);
    A.sh_logdet = p.logdet + bs;
    A.sh_yCy = p.yCy + bs;
    A.sh_ww = p.ww + bs;
    A.sh_lev_status = p.lev_status + bs;
  }
  Driver<WaveTeam> drv(*prm, S, A);
  drv.step();
  if (threadIdx.x == 0) {
    p.st[b] = S;
    if (pass == 0 && S.phase != PH_DONE) atomicAdd(p.notdone, 1);
    // this thread's own store of the request bits, read back in order
    const int32_t r = __atomic_load_n(p.req + b, __ATOMIC_RELAXED);
    if (p.req_host) p.req_host[b] = r;
    if (p.kev_host) p.kev_host[b] = __atomic_load_n(p.K_e + b, __ATOMIC_RELAXED);
    if (p.req2) {
      // a grid sweep at the point just evaluated runs in this round's second stage
      const int32_t r2 = (pass == 0 && (r & REQ_GRID) && !(r & REQ_EVAL)) ? r : 0;
      p.req2[b] = r2;
      if (p.req2_host && pass == 0) p.req2_host[b] = r2;
    }
  }
}

// ||y||^2 per instance and the initial state (phase START); with a list,
// block i initialises instance list[i] only.
template <typename YT>
__global__ __launch_bounds__(256) void k_init_state(const InstInfo* __restrict__ info,
                                                    const YT* __restrict__ y,
                                                    DrvState* __restrict__ st,
                                                    int32_t* __restrict__ req,
                                                    const int32_t* __restrict__ list, Vecs vv) {
  __shared__ double red[4];
  const int b = list ? list[blockIdx.x] : blockIdx.x;
  const InstInfo in = info[b];
  double acc[1] = {0.0};
  // the observed samples: N at off, or (incomplete observations) nobs at obsoff
  const int ny = in.nobs > 0 ? in.nobs : in.N;
  const int64_t yo = in.nobs > 0 ? in.obsoff : in.off;
  for (int gv = 0; gv < vv.G; ++gv) {
    const YT* yb = y + gv * vv.ystride + yo;
    for (int i = threadIdx.x; i < ny; i += 256) {
      const double re = (double)yb[i].x, im = (double)yb[i].y;
      acc[0] = fma(re, re, fma(im, im, acc[0]));
    }
  }
  block_sum<256, 1>(acc, red);
  if (threadIdx.x == 0) {
    DrvState s = {};
    s.phase = PH_START;
    // the energy per vector (sum over the vectors / G; G = 1: ||y||^2)
    s.yy = vv.G == 1 ? acc[0] : acc[0] / (double)vv.G;
    st[b] = s;
    req[b] = 0;
  }
}

// tw[k] = exp(-j 2 pi k / 2^logtw) for k < 2^(logtw-1) (natural order), and the
// stage-major table tws[h + pos] = exp(-j 2 pi pos / 2h) for h = 1, 2, 4, ...
__global__ void k_twiddles(cd* tw64, cf* tw32, cd* tws64, cf* tws32, int logtw) {
  const int64_t n = (int64_t)1 << logtw;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    if (k < n / 2) {
      const cd e = cis_frac(k, n);
      tw64[k] = cd{e.x, -e.y};
      tw32[k] = cf{(float)e.x, (float)-e.y};
    }
    if (k >= 1) {
      int64_t h = 1;
      while ((h << 1) <= k) h <<= 1;
      const cd e = cis_frac(k - h, 2 * h);
      tws64[k] = cd{e.x, -e.y};
      tws32[k] = cf{(float)e.x, (float)-e.y};
    } else {
      tws64[0] = cd{1.0, 0.0};
      tws32[0] = cf{1.0f, 0.0f};
    }
  }
}

__global__ void k_zero_i32(int32_t* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

hipError_t launch_driver(const InstInfo* info, const DrvParams* prm, DrvPools pools, int B,
                         hipStream_t st, int pass) {
  hipLaunchKernelGGL(k_driver, dim3(B), dim3(64), 0, st, info, prm, pools, B, pass);
  return hipGetLastError();
}

hipError_t launch_init_state(const InstInfo* info, const void* y, int ydtype, DrvState* st,
                             int32_t* req, int B, hipStream_t s, const int32_t* list, Vecs vv) {
  if (B <= 0) return hipSuccess;
  if (ydtype == 1)
    hipLaunchKernelGGL(k_init_state<cd>, dim3(B), dim3(256), 0, s, info, (const cd*)y, st, req,
                       list, vv);
  else
    hipLaunchKernelGGL(k_init_state<cf>, dim3(B), dim3(256), 0, s, info, (const cf*)y, st, req,
                       list, vv);
  return hipGetLastError();
}

// Every instance idle: phase DONE, no request (the state of a free slot).
__global__ void k_slots_idle(DrvState* __restrict__ st, int32_t* __restrict__ req, int B) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x) {
    DrvState s = {};
    s.phase = PH_DONE;
    s.done = 1;
    st[b] = s;
    req[b] = 0;
  }
}

// Pack the outputs of the instances in list[0..n) (component arrays at
// koff[i]): record i and, from comp[doff[i]], theta[K], gamma[K], then alpha
// as K interleaved pairs.
__global__ __launch_bounds__(256) void k_gather_results(
    const int32_t* __restrict__ list, const int64_t* __restrict__ doff, int n,
    const int64_t* __restrict__ koff, const int64_t* __restrict__ oK,
    const double* __restrict__ otheta, const cd* __restrict__ oalpha,
    const double* __restrict__ ogamma, const double* __restrict__ obeta,
    const double* __restrict__ ozeta, const double* __restrict__ oobj,
    const int32_t* __restrict__ oiters, const int32_t* __restrict__ oevals,
    const int32_t* __restrict__ ostatus, SlotResult* __restrict__ res,
    double* __restrict__ comp) {
  const int i = blockIdx.x;
  if (i >= n) return;
  const int b = list[i];
  const int64_t K = oK[b];
  if (threadIdx.x == 0) {
    SlotResult r;
    r.K = K;
    r.beta = obeta[b];
    r.zeta = ozeta[b];
    r.obj = oobj[b];
    r.iters = oiters[b];
    r.evals = oevals[b];
    r.status = ostatus[b];
    r.slot = b;
    res[i] = r;
  }
  double* dst = comp + doff[i];
  const int64_t ko = koff[i];
  for (int64_t k = threadIdx.x; k < K; k += blockDim.x) {
    dst[k] = otheta[ko + k];
    dst[K + k] = ogamma[ko + k];
    const cd a = oalpha[ko + k];
    dst[2 * K + 2 * k] = a.x;
    dst[2 * K + 2 * k + 1] = a.y;
  }
}

hipError_t launch_gather_results(const int32_t* list, const int64_t* doff, int n,
                                 const int64_t* koff, const int64_t* oK, const double* otheta,
                                 const cd* oalpha, const double* ogamma, const double* obeta,
                                 const double* ozeta, const double* oobj, const int32_t* oiters,
                                 const int32_t* oevals, const int32_t* ostatus, SlotResult* res,
                                 double* comp, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_results, dim3(n), dim3(256), 0, s, list, doff, n, koff, oK, otheta,
                     oalpha, ogamma, obeta, ozeta, oobj, oiters, oevals, ostatus, res, comp);
  return hipGetLastError();
}

// Admission of newly submitted instances, one block per record: the slot's
// tables from pinned host memory (read through its device mapping) into the
// device tables, and its signal into the pool, as 8-byte words.
__device__ __forceinline__ void copy_words(void* __restrict__ dst, const void* __restrict__ src,
                                           int64_t bytes) {
  const uint64_t* s = static_cast<const uint64_t*>(src);
  uint64_t* d = static_cast<uint64_t*>(dst);
  for (int64_t w = threadIdx.x; w < bytes / 8; w += blockDim.x) d[w] = s[w];
}

__global__ __launch_bounds__(256) void k_admit(const AdmitRec* __restrict__ recs, int n,
                                               const InstInfo* __restrict__ hinfo,
                                               const SepCoef* __restrict__ hcoef,
                                               const SchurLayout* __restrict__ hlay,
                                               const int64_t* __restrict__ hkoff,
                                               InstInfo* __restrict__ dinfo,
                                               SepCoef* __restrict__ dcoef,
                                               SchurLayout* __restrict__ dlay,
                                               int64_t* __restrict__ dkoff, char* __restrict__ ypool) {
  const int i = blockIdx.x;
  if (i >= n) return;
  const AdmitRec r = recs[i];
  const int b = r.slot;
  copy_words(dinfo + b, hinfo + b, sizeof(InstInfo));
  copy_words(dcoef + b, hcoef + b, sizeof(SepCoef));
  if (hlay) copy_words(dlay + b, hlay + b, sizeof(SchurLayout));
  if (threadIdx.x == 0) dkoff[b] = hkoff[b];
  if (r.src) copy_words(ypool + r.dst_bytes, r.src, r.bytes);
}

hipError_t launch_admit(const AdmitRec* recs, int n, const InstInfo* hinfo, const SepCoef* hcoef,
                        const SchurLayout* hlay, const int64_t* hkoff, InstInfo* dinfo,
                        SepCoef* dcoef, SchurLayout* dlay, int64_t* dkoff, void* ypool,
                        hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_admit, dim3(n), dim3(256), 0, s, recs, n, hinfo, hcoef, hlay, hkoff, dinfo,
                     dcoef, dlay, dkoff, static_cast<char*>(ypool));
  return hipGetLastError();
}

hipError_t launch_slots_idle(DrvState* st, int32_t* req, int B, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_slots_idle, dim3((B + 255) / 256), dim3(256), 0, s, st, req, B);
  return hipGetLastError();
}

// One workgroup, one thread per shadow slot and per instance (nsh <= 1024):
// the free slots and the wishes are ranked by block-wide prefix counts, the
// k-th wish takes the k-th free slot, and the shadows without a grant take the
// remaining slots in order.
constexpr int GRANT_NT = 1024;
constexpr int SPEC_MAX = GRANT_NT;

// exclusive prefix count of f over the workgroup (thread order), and the total
__device__ __forceinline__ int grant_scan(bool f, int* s_w, int& total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const unsigned long long m = __ballot(f);
  const int before = __popcll(m & ((1ull << lane) - 1ull));
  __syncthreads();
  if (lane == 0) s_w[wv] = __popcll(m);
  __syncthreads();
  int base = 0, tot = 0;
  for (int i = 0; i < GRANT_NT / 64; ++i) {
    if (i < wv) base += s_w[i];
    tot += s_w[i];
  }
  total = tot;
  return base + before;
}

__global__ __launch_bounds__(GRANT_NT) void k_spec_grant(int32_t* __restrict__ req,
                                                         int32_t* __restrict__ wish,
                                                         int32_t* __restrict__ ord, int nsh,
                                                         int ncu) {
  __shared__ int s_w[GRANT_NT / 64];
  __shared__ int s_by_rank[SPEC_MAX];
  __shared__ int s_other[SPEC_MAX];
  const int j = threadIdx.x;  // slot j and instance j
  const bool in = j < nsh;
  // slot j: the CU slot of shadow workgroup nsh + j, and the instance there
  const int c = in ? (nsh + j) % ncu : 0;
  const bool fr = in && (c >= nsh || !(req[ord[c]] & REQ_EVAL));
  const bool prim = in && (req[j] & REQ_EVAL);
  const bool wi = in && wish[j] != 0;
  int nprim, nfree, nwish;
  (void)grant_scan(prim, s_w, nprim);
  const int rf = grant_scan(fr, s_w, nfree);
  const int rw = grant_scan(wi, s_w, nwish);
  // only while at most half the CUs evaluate (measured: with more, the
  // shadows of a round can still land behind a busy CU and double it)
  const int ngr = nprim > ncu / 2 ? 0 : (nwish < nfree ? nwish : nfree);
  const bool gr = wi && rw < ngr;
  if (gr) s_by_rank[rw] = j;
  // the slots without a granted shadow, and the shadows without a grant
  const bool u = in && !(fr && rf < ngr);
  const bool v = in && !gr;
  int nu, nv;
  const int ru = grant_scan(u, s_w, nu);
  const int rv = grant_scan(v, s_w, nv);
  if (v) s_other[rv] = j;
  __syncthreads();
  if (in) {
    const int owner = (fr && rf < ngr) ? s_by_rank[rf] : s_other[ru];
    ord[nsh + j] = nsh + owner;
    req[nsh + j] = gr ? REQ_EVAL : 0;
    wish[j] = 0;
  }
}

hipError_t launch_spec_grant(int32_t* req, int32_t* wish, int32_t* ord, int nsh, int ncu,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_spec_grant, dim3(1), dim3(GRANT_NT), 0, st, req, wish, ord, nsh, ncu);
  return hipGetLastError();
}

hipError_t launch_twiddles(cd* tw64, cf* tw32, cd* tws64, cf* tws32, int logtw, hipStream_t st) {
  hipLaunchKernelGGL(k_twiddles, dim3(256), dim3(256), 0, st, tw64, tw32, tws64, tws32, logtw);
  return hipGetLastError();
}

hipError_t launch_zero_i32(int32_t* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, p, n);
  return hipGetLastError();
}

}  // namespace sfls
