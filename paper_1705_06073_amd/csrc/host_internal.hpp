// Host-side internals shared by the C-ABI translation units (abi.hip,
// server.hip): the context, workspace helpers, and the planning of sizes that
// the kernels read from InstInfo / SchurLayout.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "k_launch.hpp"
#include "sfls.h"

struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
};

enum KernelId { KID_GEN = 0, KID_FACTOR, KID_REFINE, KID_APPLY, KID_OMEGA, KID_GRID, KID_SELECT,
                KID_ACTIVE, KID_DRIVER, KID_COUNT };

struct sfls_ctx {
  int device = 0;
  std::string err;
  sfls::cd* tw64 = nullptr;
  sfls::cf* tw32 = nullptr;
  sfls::cd* tws64 = nullptr;  // stage-major FFT twiddles
  sfls::cf* tws32 = nullptr;
  int logtw = 17;
  std::map<std::string, DevBuf> bufs;
  int32_t* host_req = nullptr;  // pinned per-instance request words, two sets (req, req2, K)
  int64_t host_req_n = 0;
  int32_t timing = 0;  // 0 off, 1 every kernel of a round, 2 the recursion only
  int32_t factor_algo = 0;  // sfls_factor_algo
  int32_t nufft_mode = 0;   // sfls_nufft_mode
  int32_t spec = 1;         // shadow evaluations of line-search trials (sfls_set_speculation)
  int32_t ncu = 256;        // compute units of the device (workgroup slots the shadows may take)
  // per round parity, stage (first, second) and kernel: start and stop
  hipEvent_t ev[8 * KID_COUNT] = {};
  sfls_kernel_stat kst[KID_COUNT] = {};
  sfls_run_stats last = {};
  std::vector<double> timeline;
  hipStream_t upload = nullptr;  // admission copies of the servers on this context
  hipEvent_t ev_rounds[2] = {};  // end of an estimate round, by parity (request words on the host)
  int32_t schur_lds_f = sfls::SCH_LDS_F;  // largest recursion transform kept in LDS
  size_t hbm_budget = 0;  // workspace limit in bytes (0: none)
  size_t ws_bytes = 0;    // workspace held
};

// Whether timing mode `mode` (sfls_set_timing) brackets kernel k with events.
inline bool times_kernel(int32_t mode, int k) {
  return mode == 1 || (mode == 2 && k == KID_FACTOR);
}

namespace sfls_host {

using sfls::cd;
using sfls::cf;

sfls_status fail(sfls_ctx* ctx, sfls_status s, const char* fmt, ...);

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return sfls_host::fail(ctx, SFLS_EDEVICE, "%s failed: %s", #expr,                      \
                             hipGetErrorString(e_));                                         \
  } while (0)

// Largest sizes of a batch.
struct Sizes {
  int maxN = 0, maxP = 0, maxM = 0, Rmax = 1;
};
// Host checks of a ragged batch: B >= 0, n and off given, nmin <= n[b] <= SFLS_MAX_N.
sfls_status check_batch(sfls_ctx* ctx, int64_t B, const int64_t* n, const int64_t* off,
                        int64_t nmin);
// Base InstInfo: N, P, off, poff (4 P scratch per instance, plus a transform
// buffer when P exceeds the LDS transform size); ptotal = scratch elements.
std::vector<sfls::InstInfo> base_info(int64_t B, const int64_t* n, const int64_t* off, Sizes& sz,
                                      int64_t& ptotal);
hipStream_t as_stream(void* s);
// Device address of the static scratch of sfls_gs_apply_noalloc on the
// context's device (looked up once per device, at context creation).
sfls_status noalloc_init(sfls_ctx* ctx);

int ilog2_ceil(int64_t v);
// Dispatch order of a batch whose sizes differ: instance indices by
// decreasing N (stable); empty when every N is equal (identity order).
std::vector<int32_t> longest_first(int64_t B, const int64_t* n);
// Wait for an event by polling it: a blocking wait can leave the device idle
// for a scheduler wake-up between rounds, which sets the pace of the round
// loops (one host decision per round).
hipError_t spin_wait(hipEvent_t ev);
bool is_pow2(int64_t v);

// Coefficients of the separable forms of s, t, v, x for N samples.
void sep_coef(int N, sfls::SepCoef& out);

// The superfast recursion of one N flattened into actions.
struct SchurPlan {
  std::vector<sfls::SchurAct> acts;
  int32_t mmax[sfls::SCH_MAXL] = {};
  int32_t fspec[sfls::SCH_MAXL] = {};
  int nlev = 0;
};
constexpr int kSchurMinN = 256;  // AUTO: superfast Schur from this N on

// Plan of the recursion for N samples (no actions for N = 1).
SchurPlan schur_plan(int64_t N);
// Algorithmic FP64 flops of one factorisation by `P`.
double schur_flops(const SchurPlan& P);
// Per-instance scratch layout of `P` (offsets from the instance's scratch
// start; scr_off, act_off and Fmax are left to the caller).  Returns the
// scratch size in complex elements; *fm receives the LDS transform size the
// plan needs.
int64_t schur_layout(const SchurPlan& P, sfls::SchurLayout& L, int* fm,
                     int lds_f = sfls::SCH_LDS_F);

// Factorisation the context uses for a batch whose largest N is maxN.
bool use_schur(const sfls_ctx* ctx, int maxN);
constexpr int kLevinsonMaxN = 4096;  // the Levinson kernel keeps vectors in registers
// Grid sub-FFT size M = min(2^ceil(log2 N), cap), cap set by the grid's precision.
void cap_grid_m(sfls::InstInfo& in, int precision);
// Conversion of the public parameters into the driver's.
sfls::DrvParams drv_params(const sfls_params& p);
// Range checks of sfls_params.
bool params_valid(const sfls_params& p);

}  // namespace sfls_host
