// Serving by continuous batching: the round loop of sfls_estimate run over a
// pool of request slots that fill and drain while rounds continue.
//
// Memory: every per-request array of the round loop lives in one of a few
// device pools indexed by the request's offsets (InstInfo / SchurLayout).  A
// request of length N takes one buddy block of 2^ceil(log2 max(N, 64))
// samples; each pool holds a fixed number of elements per sample (the
// convolution scratch 11, the grid 2^round(log2 L_mult), the recursion's
// scratch the largest ratio over the supported sizes, the component arrays
// 2^-kcap_shift), so one buddy offset places the request in every pool.
// Admission is the buddy allocation: a request is admitted when a block of
// its order is free, i.e. by its device-memory footprint.
//
// Per-slot arrays (driver state, request bits, scalars, candidates) are
// indexed by the slot.  Free slots hold phase DONE and no request bits, so
// every kernel of a round returns at once for them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <set>
#include <vector>

#include "host_internal.hpp"

using namespace sfls;
using namespace sfls_host;

static_assert(sizeof(sfls_server_config) == 40, "sfls_server_config layout is part of the ABI");
static_assert(sizeof(sfls_result) == 88, "sfls_result layout is part of the ABI");
static_assert(sizeof(sfls_server_stats) == 72, "sfls_server_stats layout is part of the ABI");

namespace {

constexpr int64_t kUnitMin = 64;  // smallest pool block, in samples
constexpr int64_t kConvPerSample = 11;  // 4 P + padded(P) <= 11 * block for P <= 2 * block
constexpr int kMaxSlots = 65536;

// Buddy allocator over 2^top blocks of kUnitMin samples.
struct Buddy {
  int top = 0;
  std::vector<std::set<int64_t>> freel;  // free block starts (in kUnitMin blocks) per order
  void init(int top_order) {
    top = top_order;
    freel.assign((size_t)top + 1, std::set<int64_t>{});
    freel[(size_t)top].insert(0);
  }
  int64_t alloc(int order) {
    int o = order;
    while (o <= top && freel[(size_t)o].empty()) ++o;
    if (o > top) return -1;
    const int64_t b = *freel[(size_t)o].begin();
    freel[(size_t)o].erase(freel[(size_t)o].begin());
    while (o > order) {
      --o;
      freel[(size_t)o].insert(b + ((int64_t)1 << o));
    }
    return b;
  }
  void release(int64_t b, int order) {
    int o = order;
    while (o < top) {
      const int64_t buddy = b ^ ((int64_t)1 << o);
      auto it = freel[(size_t)o].find(buddy);
      if (it == freel[(size_t)o].end()) break;
      freel[(size_t)o].erase(it);
      b = std::min(b, buddy);
      ++o;
    }
    freel[(size_t)o].insert(b);
  }
};

enum SlotState : int8_t { SLOT_FREE = 0, SLOT_ADMITTED = 1, SLOT_RUNNING = 2 };

struct Slot {
  SlotState state = SLOT_FREE;
  int order = 0;
  int64_t block = 0;  // buddy block start (kUnitMin units)
  uint64_t tag = 0;
  double t_submit = 0.0;
};

struct PlanEntry {
  int64_t act_off = 0;
  SchurLayout lay{};
  int64_t scratch = 0;  // complex elements
  int fm = 0;
  double flops = 0.0;   // algorithmic FP64 flops of one factorisation
};

struct Result {
  sfls_result r{};
  std::vector<double> comp;  // theta[K], gamma[K], alpha[2K]
};

template <typename T>
hipError_t dalloc(T** p, size_t count, std::vector<void*>& owned) {
  *p = nullptr;
  void* v = nullptr;
  hipError_t e = hipMalloc(&v, std::max<size_t>(count, 1) * sizeof(T));
  if (e == hipSuccess) {
    owned.push_back(v);
    *p = static_cast<T*>(v);
  }
  return e;
}

// Pinned host memory, fine-grained (coherent): kernels read and write some of
// these buffers directly, and the host reads what they wrote after an event.
template <typename T>
hipError_t halloc(T** p, size_t count, std::vector<void*>& owned) {
  *p = nullptr;
  void* v = nullptr;
  hipError_t e = hipHostMalloc(&v, std::max<size_t>(count, 1) * sizeof(T),
                               hipHostMallocMapped | hipHostMallocCoherent);
  if (e == hipSuccess) {
    owned.push_back(v);
    *p = static_cast<T*>(v);
  }
  return e;
}

int order_of(int64_t blocks) {  // blocks: a power of two
  int o = 0;
  while (((int64_t)1 << o) < blocks) ++o;
  return o;
}

}  // namespace

struct sfls_server {
  sfls_ctx* ctx = nullptr;
  sfls_server_config cfg{};
  sfls_params prm{};
  bool own_stream = false;
  hipStream_t st = nullptr;   // rounds
  hipStream_t up = nullptr;   // admission copies (the context's upload stream)
  hipEvent_t ev = nullptr;    // end of the round in flight
  hipEvent_t ev_res = nullptr;  // end of the result gather in flight
  bool schur = false;
  int Fmax = 0;               // LDS transform size of the recursion (fixed per server)
  int lds_f = SCH_LDS_F;      // largest recursion transform in LDS (fixed per server)
  int64_t fL = 1, fS = 1;     // grid and recursion-scratch elements per pool sample
  int kshift = 2;
  int Rmax = 1;
  int cc = 0;                 // candidate entries per slot
  size_t ysz = 8, esz = 4;
  uint64_t bpu = 0;           // bytes per pool sample
  int64_t units = 0;          // pool samples
  uint64_t bytes_reserved = 0;
  Buddy buddy;
  std::vector<Slot> slots;
  std::set<int> free_slots;
  int hw = 0;                 // 1 + highest occupied slot index
  std::vector<int> admitted;  // slots admitted since the last launch
  std::deque<Result> done;
  bool in_flight = false;
  std::chrono::steady_clock::time_point t0, t_launch;
  sfls_server_stats stats{};
  // per-kernel HIP events of the round in flight (when the context times)
  hipEvent_t tev[4 * KID_COUNT] = {};  // per kernel: start/stop of the first and second stage
  bool tlaunched[KID_COUNT] = {}, tlaunched2[KID_COUNT] = {};
  int32_t tmode = 0;
  double tflops[KID_COUNT] = {}, tbytes[KID_COUNT] = {};
  bool timed = false;
  std::vector<double> slot_flops;  // factorisation flops of each slot's request

  // device pools (offset-indexed)
  void* ypool = nullptr;
  cd *c = nullptr, *rho = nullptr, *w = nullptr, *rf_r = nullptr, *rf_dx = nullptr;
  double* delta = nullptr;
  cd *scratch = nullptr, *oms = nullptr, *sscr = nullptr;
  void* dL = nullptr;
  DrvPools P{};
  cd *evq = nullptr, *evr = nullptr, *evu = nullptr, *evs = nullptr, *evt = nullptr,
     *evv = nullptr, *evx = nullptr;
  // per-slot
  InstInfo* dinfo = nullptr;
  SepCoef* dcoef = nullptr;
  SchurLayout* dlay = nullptr;
  int64_t* dkoff = nullptr;
  DrvParams* dprm = nullptr;
  double *logdet = nullptr, *yCy = nullptr, *ww = nullptr, *pv = nullptr;
  int64_t *failed = nullptr, *pi = nullptr;
  int32_t *lev_status = nullptr, *prefix = nullptr, *ovf = nullptr, *cand = nullptr,
          *ncand = nullptr, *notdone = nullptr;
  cd* cq = nullptr;
  double* cs = nullptr;
  // result gathering: finished slots are released when found; their outputs
  // are packed by a kernel enqueued behind the round that finished them (the
  // slot list and output offsets travel with it, so a new occupant's tables
  // cannot race it) straight into pinned host memory, read by the next poll
  int64_t* h_gkoff = nullptr;
  bool gather_pending = false;
  std::vector<Result> gathering;  // metadata of the results in flight
  // recursion action pool
  SchurAct* dacts = nullptr;
  size_t acts_cap = 0, acts_n = 0;
  std::map<int64_t, PlanEntry> plans;
  std::deque<std::vector<SchurAct>> plan_src;  // host sources of uploaded actions
  // pinned host mirrors
  InstInfo* h_info = nullptr;
  SepCoef* h_coef = nullptr;
  SchurLayout* h_lay = nullptr;
  int64_t* h_koff = nullptr;
  int32_t* h_req = nullptr;
  int32_t* h_req2 = nullptr;     // second-stage grid requests of the last round (accounting)
  int32_t* h_list = nullptr;
  int32_t* h_order = nullptr;    // dispatch order of the round (lanes of uneven sizes)
  int32_t* h_newlist = nullptr;  // [2][S]: admitted since the last launch, by buffer
  AdmitRec* h_adm = nullptr;     // [2][S]
  int abuf = 0;                  // buffer that submissions fill; a launch takes it and flips
  int64_t* h_doff = nullptr;
  SlotResult* h_res = nullptr;
  double* h_comp = nullptr;
  size_t h_comp_n = 0;
  std::vector<void*> dev_owned, host_owned;
  // device addresses of the pinned buffers the kernels read or write directly
  int32_t* m_req = nullptr;
  int32_t* m_req2 = nullptr;
  int32_t* m_newlist = nullptr;
  int32_t* m_order = nullptr;
  AdmitRec* m_adm = nullptr;
  InstInfo* m_info = nullptr;
  SepCoef* m_coef = nullptr;
  SchurLayout* m_lay = nullptr;
  int64_t* m_koff = nullptr;
  int32_t* m_list = nullptr;
  int64_t* m_doff = nullptr;
  int64_t* m_gkoff = nullptr;
  SlotResult* m_res = nullptr;
  double* m_comp = nullptr;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  int64_t kcap_of(int64_t n, int64_t blk_samples) const {
    return std::min<int64_t>(n, std::max<int64_t>(1, blk_samples >> kshift));
  }
};

namespace {

// Plan of the recursion for n (cached; actions appended to the device pool).
sfls_status plan_for(sfls_server* s, int64_t n, const PlanEntry** out) {
  auto it = s->plans.find(n);
  if (it != s->plans.end()) {
    *out = &it->second;
    return SFLS_OK;
  }
  sfls_ctx* ctx = s->ctx;
  SchurPlan P = schur_plan(n);
  PlanEntry e;
  e.scratch = schur_layout(P, e.lay, &e.fm, s->lds_f);
  e.flops = schur_flops(P);
  if (e.fm > s->Fmax) return fail(ctx, SFLS_EUNSUPPORTED, "recursion plan of n = %lld needs a larger transform", (long long)n);
  const size_t na = std::max<size_t>(P.acts.size(), 1);
  if (s->acts_n + na > s->acts_cap) {
    // grow: only between rounds, the device pool is then idle
    if (s->in_flight) return SFLS_EAGAIN;
    HIP_TRY(hipStreamSynchronize(s->st));
    size_t cap = std::max<size_t>(2 * s->acts_cap, s->acts_n + na);
    SchurAct* nb = nullptr;
    if (hipMalloc(&nb, cap * sizeof(SchurAct)) != hipSuccess)
      return fail(ctx, SFLS_ENOMEM, "recursion action pool of %zu entries", cap);
    if (s->acts_n) HIP_TRY(hipMemcpy(nb, s->dacts, s->acts_n * sizeof(SchurAct), hipMemcpyDeviceToDevice));
    auto old = std::find(s->dev_owned.begin(), s->dev_owned.end(), (void*)s->dacts);
    if (old != s->dev_owned.end()) s->dev_owned.erase(old);
    if (s->dacts) (void)hipFree(s->dacts);
    s->dacts = nb;
    s->dev_owned.push_back(nb);
    s->acts_cap = cap;
  }
  s->plan_src.emplace_back(P.acts);
  if (s->plan_src.back().empty()) s->plan_src.back().push_back(SchurAct{});
  HIP_TRY(hipMemcpyAsync(s->dacts + s->acts_n, s->plan_src.back().data(), na * sizeof(SchurAct),
                         hipMemcpyHostToDevice, s->up));
  HIP_TRY(hipStreamSynchronize(s->up));
  e.act_off = (int64_t)s->acts_n;
  e.lay.act_off = e.act_off;
  e.lay.Fmax = s->Fmax;
  s->acts_n += na;
  *out = &s->plans.emplace(n, e).first->second;
  return SFLS_OK;
}

// Pool layout of a request of length n in a block of 2^order kUnitMin units
// starting at block start b; false if some array would not fit the block.
bool place(const sfls_server* s, int64_t n, int order, int64_t b, const PlanEntry* pe,
           InstInfo& in, SchurLayout& lay) {
  const int64_t blk = kUnitMin << order;  // samples
  const int64_t u0 = b * kUnitMin;
  std::memset(&in, 0, sizeof in);
  in.N = (int32_t)n;
  in.logP = ilog2_ceil(2 * n - 1 > 1 ? 2 * n - 1 : 2);
  in.P = 1 << in.logP;
  in.logM = ilog2_ceil(n);
  in.M = 1 << in.logM;
  const int64_t Lb = (int64_t)1 << (int)std::lround(std::log2(s->prm.L_mult * (double)n));
  const int64_t conv = 4 * (int64_t)in.P + (in.P > CONV_LDS_P ? (int64_t)padded(in.P) : 0);
  if (n > blk || conv > kConvPerSample * blk || Lb > s->fL * blk) return false;
  if (pe && pe->scratch > s->fS * blk) return false;
  cap_grid_m(in, s->prm.precision);
  in.L = (int32_t)Lb;
  in.R = (int32_t)(Lb / in.M);
  if (in.R > s->Rmax) return false;
  in.kcap = (int32_t)s->kcap_of(n, blk);
  in.off = u0;
  in.poff = u0 * kConvPerSample;
  in.goff = u0 * s->fL;
  in.koff = u0 >> s->kshift;
  in.ooff = 0;
  if (pe) {
    lay = pe->lay;
    lay.scr_off = u0 * s->fS;
  } else {
    std::memset(&lay, 0, sizeof lay);
  }
  return true;
}

}  // namespace

// Complete a result gather: wait for it (it is short and runs right behind
// the round that found the results) and move the packed outputs into the
// result queue.
static sfls_status finish_gather(sfls_server* s) {
  if (!s->gather_pending) return SFLS_OK;
  sfls_ctx* ctx = s->ctx;
  HIP_TRY(spin_wait(s->ev_res));
  for (size_t i = 0; i < s->gathering.size(); ++i) {
    const SlotResult& r = s->h_res[i];
    Result& out = s->gathering[i];
    out.r.K = r.K;
    out.r.beta = r.beta;
    out.r.zeta = r.zeta;
    out.r.objective = r.obj;
    out.r.iters = r.iters;
    out.r.evals = r.evals;
    out.r.status = r.status;
    const double* src = s->h_comp + s->h_doff[i];
    out.comp.assign(src, src + 4 * r.K);
    s->done.push_back(std::move(out));
  }
  s->gathering.clear();
  s->gather_pending = false;
  return SFLS_OK;
}

extern "C" {

void sfls_server_config_default(sfls_server_config* cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof *cfg);
  cfg->max_n = SFLS_MAX_N;
  cfg->max_slots = 1024;
  cfg->ydtype = SFLS_C64;
  cfg->hbm_bytes = (uint64_t)8 << 30;
  cfg->kcap_shift = 0;
  cfg->stream = nullptr;
}

sfls_status sfls_server_destroy(sfls_server* s) {
  if (!s) return SFLS_OK;
  (void)hipSetDevice(s->ctx->device);
  if (s->st) (void)hipStreamSynchronize(s->st);
  if (s->up) (void)hipStreamSynchronize(s->up);
  for (void* p : s->dev_owned) (void)hipFree(p);
  for (void* p : s->host_owned) (void)hipHostFree(p);
  if (s->ev) (void)hipEventDestroy(s->ev);
  if (s->ev_res) (void)hipEventDestroy(s->ev_res);
  for (auto& e : s->tev)
    if (e) (void)hipEventDestroy(e);
  if (s->own_stream && s->st) (void)hipStreamDestroy(s->st);
  delete s;
  return SFLS_OK;
}

sfls_status sfls_server_create(sfls_ctx* ctx, const sfls_server_config* cfg_in,
                               const sfls_params* params, sfls_server** out) {
  if (!ctx || !out) return SFLS_EINVAL;
  *out = nullptr;
  ctx->err.clear();
  sfls_server_config cfg;
  if (cfg_in) cfg = *cfg_in; else sfls_server_config_default(&cfg);
  sfls_params p;
  if (params) p = *params; else sfls_params_default(&p);
  if (!params_valid(p)) return fail(ctx, SFLS_EINVAL, "invalid sfls_params");
  if (cfg.max_n < 2 || cfg.max_n > SFLS_MAX_N)
    return fail(ctx, cfg.max_n > SFLS_MAX_N ? SFLS_EUNSUPPORTED : SFLS_EINVAL,
                "max_n = %lld outside 2..%d", (long long)cfg.max_n, SFLS_MAX_N);
  if (cfg.max_slots < 1 || cfg.max_slots > kMaxSlots)
    return fail(ctx, SFLS_EINVAL, "max_slots = %d outside 1..%d", cfg.max_slots, kMaxSlots);
  if (cfg.ydtype != SFLS_C64 && cfg.ydtype != SFLS_C128) return fail(ctx, SFLS_EINVAL, "bad ydtype");
  if (cfg.kcap_shift < 0 || cfg.kcap_shift > 6) return fail(ctx, SFLS_EINVAL, "kcap_shift outside 0..6");
  (void)hipSetDevice(ctx->device);

  sfls_server* s = new sfls_server();
  s->ctx = ctx;
  s->cfg = cfg;
  s->prm = p;
  s->t0 = std::chrono::steady_clock::now();
  s->kshift = cfg.kcap_shift;
  s->ysz = cfg.ydtype == SFLS_C128 ? 16 : 8;
  s->esz = p.precision == SFLS_FP64 ? 8 : 4;
  s->cc = p.cand_cap + 1;
  s->schur = use_schur(ctx, (int)cfg.max_n);
  auto bail = [&](sfls_status code) {
    sfls_server_destroy(s);
    return code;
  };
  if (!s->schur && cfg.max_n > kLevinsonMaxN)
    return bail(fail(ctx, SFLS_EUNSUPPORTED, "the Levinson recursion supports n <= %d", kLevinsonMaxN));
  const int64_t top_blk = std::max<int64_t>(kUnitMin, (int64_t)1 << ilog2_ceil(cfg.max_n));
  // grid elements per sample: L of a power-of-two block is 2^round(log2 L_mult) per sample
  {
    const int64_t Lt = (int64_t)1 << (int)std::lround(std::log2(p.L_mult * (double)top_blk));
    s->fL = std::max<int64_t>(1, Lt / top_blk);
    int64_t rmax = 1;  // grid residues R = L / M over every admissible length
    for (int64_t n = 2; n <= cfg.max_n; ++n) {
      InstInfo t{};
      t.logM = ilog2_ceil(n);
      t.M = 1 << t.logM;
      cap_grid_m(t, p.precision);
      const int64_t Lb = (int64_t)1 << (int)std::lround(std::log2(p.L_mult * (double)n));
      rmax = std::max<int64_t>(rmax, Lb / t.M);
    }
    s->Rmax = (int)rmax;
  }
  // recursion: scratch per sample and the server's transform size
  s->Fmax = 64;
  s->fS = 1;
  s->lds_f = ctx->schur_lds_f;
  if (s->schur) {
    for (int64_t blk = kUnitMin; blk <= top_blk; blk *= 2) {
      SchurPlan P = schur_plan(blk);
      SchurLayout L;
      int fm = 64;
      const int64_t o = schur_layout(P, L, &fm, s->lds_f);
      s->Fmax = std::max(s->Fmax, fm);
      s->fS = std::max<int64_t>(s->fS, (o + blk - 1) / blk);
    }
  }
  const int J = p.lbfgs_J;
  const double kbytes = 4 * 8 + 4 * 16 + 2.0 * 2 * J * 8 + 7 * 16 + 2 * 8 + 16;  // per component
  s->bpu = (uint64_t)(s->ysz + 5 * 16 + 8 + 2 * kConvPerSample * 16 + s->fL * s->esz + s->fS * 16 +
                      std::ceil(kbytes / (double)((int64_t)1 << s->kshift)));
  const int64_t S = cfg.max_slots;
  const uint64_t slot_bytes =
      (uint64_t)S * (sizeof(InstInfo) + sizeof(SepCoef) + sizeof(SchurLayout) + sizeof(DrvState) +
                     8 * 16 + (uint64_t)s->Rmax * 16 + 2 * (uint64_t)J * 8 +
                     (uint64_t)s->cc * (4 + 16 + 8 + 8 + 8 + 4) + sizeof(SlotResult) + 20);
  if (cfg.hbm_bytes <= slot_bytes)
    return bail(fail(ctx, SFLS_EINVAL, "hbm_bytes below the per-slot arrays (%llu bytes)",
                     (unsigned long long)slot_bytes));
  int64_t units = kUnitMin;
  while ((uint64_t)(2 * units) * s->bpu <= cfg.hbm_bytes - slot_bytes) units *= 2;
  if ((uint64_t)units * s->bpu > cfg.hbm_bytes - slot_bytes || units < top_blk)
    return bail(fail(ctx, SFLS_EINVAL,
                     "hbm_bytes = %llu holds no request of max_n = %lld (needs %llu bytes)",
                     (unsigned long long)cfg.hbm_bytes, (long long)cfg.max_n,
                     (unsigned long long)(slot_bytes + (uint64_t)top_blk * s->bpu)));
  s->units = units;
  s->buddy.init(order_of(units / kUnitMin));
  s->slots.assign((size_t)S, Slot{});
  s->slot_flops.assign((size_t)S, 0.0);
  for (int i = 0; i < S; ++i) s->free_slots.insert(i);

  // streams and events (default priority)
  if (cfg.stream) {
    s->st = reinterpret_cast<hipStream_t>(cfg.stream);
  } else {
    if (hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking) != hipSuccess)
      return bail(fail(ctx, SFLS_EDEVICE, "stream creation failed"));
    s->own_stream = true;
  }
  // one upload stream per context: every stream of a process takes one of its
  // few hardware queues, and the round streams should not share them
  if (!ctx->upload && hipStreamCreateWithFlags(&ctx->upload, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(ctx, SFLS_EDEVICE, "stream creation failed"));
  s->up = ctx->upload;
  if (hipEventCreateWithFlags(&s->ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&s->ev_res, hipEventDisableTiming) != hipSuccess)
    return bail(fail(ctx, SFLS_EDEVICE, "stream/event creation failed"));

  auto& D = s->dev_owned;
  const size_t U = (size_t)units, K = (size_t)(units >> s->kshift);
  bool ok = true;
#define DA(ptr, cnt) ok = ok && dalloc(&(ptr), (size_t)(cnt), D) == hipSuccess
  void* yp = nullptr;
  ok = ok && hipMalloc(&yp, U * s->ysz) == hipSuccess;
  if (yp) D.push_back(yp);
  s->ypool = yp;
  DA(s->c, U); DA(s->rho, U); DA(s->w, U); DA(s->rf_r, U); DA(s->rf_dx, U); DA(s->delta, U);
  DA(s->scratch, U * kConvPerSample); DA(s->oms, U * kConvPerSample);
  if (s->schur) DA(s->sscr, U * (size_t)s->fS);
  void* dl = nullptr;
  ok = ok && hipMalloc(&dl, U * (size_t)s->fL * s->esz) == hipSuccess;
  if (dl) D.push_back(dl);
  s->dL = dl;
  DrvPools& P = s->P;
  DA(P.st, S);
  DA(P.th, K); DA(P.ga, K); DA(P.th_e, K); DA(P.ga_e, K);
  DA(P.g, 2 * K); DA(P.d, 2 * K); DA(P.gt, 2 * K); DA(P.q_save, 2 * K);
  DA(P.Sm, (size_t)J * 2 * K); DA(P.Ym, (size_t)J * 2 * K);
  DA(P.rhom, (size_t)J * S); DA(P.am, (size_t)J * S);
  DA(P.K_e, S); DA(P.req, S); DA(P.req2, S); DA(P.beta_e, S); DA(P.gbar_e, S); DA(P.zeta_e, S);
  DA(s->evq, K); DA(s->evr, K); DA(s->evu, K); DA(s->evs, K); DA(s->evt, K); DA(s->evv, K);
  DA(s->evx, K);
  DA(s->logdet, S); DA(s->yCy, S); DA(s->ww, S); DA(s->failed, S); DA(s->lev_status, S);
  DA(s->prefix, S + 1); DA(s->ovf, S); DA(s->ncand, S); DA(s->notdone, 1);
  DA(s->pv, (size_t)S * s->Rmax); DA(s->pi, (size_t)S * s->Rmax);
  DA(s->cand, (size_t)S * s->cc); DA(s->cq, (size_t)S * s->cc); DA(s->cs, (size_t)S * s->cc);
  DA(P.cbuf_dl, (size_t)S * s->cc); DA(P.cbuf_gh, (size_t)S * s->cc); DA(P.cbuf_l, (size_t)S * s->cc);
  cd* oalpha = nullptr;
  double *otheta = nullptr, *ogamma = nullptr, *obeta = nullptr, *ozeta = nullptr, *oobj = nullptr;
  int64_t* oK = nullptr;
  int32_t *oit = nullptr, *oev = nullptr, *ost = nullptr;
  DA(otheta, K); DA(ogamma, K); DA(oalpha, K);
  DA(oK, S); DA(obeta, S); DA(ozeta, S); DA(oobj, S); DA(oit, S); DA(oev, S); DA(ost, S);
  DA(s->dinfo, S); DA(s->dcoef, S); DA(s->dlay, S); DA(s->dkoff, S); DA(s->dprm, 1);
  if (s->schur) {
    s->acts_cap = 16384;
    DA(s->dacts, s->acts_cap);
  }
#undef DA
  if (!ok) return bail(fail(ctx, SFLS_ENOMEM, "server pools (%llu bytes) not available",
                            (unsigned long long)cfg.hbm_bytes));
  auto& H = s->host_owned;
#define HA(ptr, cnt) ok = ok && halloc(&(ptr), (size_t)(cnt), H) == hipSuccess
  HA(s->h_info, S); HA(s->h_coef, S); HA(s->h_lay, S); HA(s->h_koff, S); HA(s->h_req, S);
  HA(s->h_list, S); HA(s->h_newlist, 2 * S); HA(s->h_adm, 2 * S); HA(s->h_doff, S);
  HA(s->h_gkoff, S); HA(s->h_res, S); HA(s->h_order, S); HA(s->h_req2, S);
#undef HA
  if (!ok) return bail(fail(ctx, SFLS_ENOMEM, "pinned host mirrors"));
  std::memset(s->h_req, 0, (size_t)S * sizeof(int32_t));
  std::memset(s->h_req2, 0, (size_t)S * sizeof(int32_t));
  if (hipHostGetDevicePointer((void**)&s->m_req, s->h_req, 0) != hipSuccess ||
      hipHostGetDevicePointer((void**)&s->m_newlist, s->h_newlist, 0) != hipSuccess ||
      hipHostGetDevicePointer((void**)&s->m_adm, s->h_adm, 0) != hipSuccess ||
      hipHostGetDevicePointer((void**)&s->m_info, s->h_info, 0) != hipSuccess ||
      hipHostGetDevicePointer((void**)&s->m_coef, s->h_coef, 0) != hipSuccess ||
      hipHostGetDevicePointer((void**)&s->m_lay, s->h_lay, 0) != hipSuccess ||
      hipHostGetDevicePointer((void**)&s->m_koff, s->h_koff, 0) != hipSuccess ||
      hipHostGetDevicePointer((void**)&s->m_list, s->h_list, 0) != hipSuccess ||
      hipHostGetDevicePointer((void**)&s->m_doff, s->h_doff, 0) != hipSuccess ||
      hipHostGetDevicePointer((void**)&s->m_gkoff, s->h_gkoff, 0) != hipSuccess ||
      hipHostGetDevicePointer((void**)&s->m_res, s->h_res, 0) != hipSuccess ||
      hipHostGetDevicePointer((void**)&s->m_order, s->h_order, 0) != hipSuccess ||
      hipHostGetDevicePointer((void**)&s->m_req2, s->h_req2, 0) != hipSuccess)
    return bail(fail(ctx, SFLS_EDEVICE, "device addresses of the pinned mirrors"));
  P.ev_q = s->evq; P.ev_r = s->evr; P.ev_u = s->evu; P.ev_s = s->evs; P.ev_t = s->evt;
  P.ev_v = s->evv; P.ev_x = s->evx; P.logdet = s->logdet; P.yCy = s->yCy; P.ww = s->ww;
  P.lev_status = s->lev_status; P.cand = s->cand; P.ncand = s->ncand; P.cand_q = s->cq;
  P.cand_s = s->cs; P.out_K = oK; P.out_theta = otheta; P.out_alpha = oalpha;
  P.out_gamma = ogamma; P.out_beta = obeta; P.out_zeta = ozeta; P.out_obj = oobj;
  P.out_iters = oit; P.out_evals = oev; P.out_status = ost; P.out_koff = s->dkoff;
  P.notdone = s->notdone;
  P.req_host = s->m_req;
  P.req2_host = s->m_req2;
  const DrvParams dp = drv_params(p);
  std::vector<InstInfo> zinfo((size_t)S);
  std::memset(zinfo.data(), 0, zinfo.size() * sizeof(InstInfo));
  if (hipMemcpy(s->dprm, &dp, sizeof dp, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(s->dinfo, zinfo.data(), zinfo.size() * sizeof(InstInfo), hipMemcpyHostToDevice) !=
          hipSuccess ||
      launch_slots_idle(P.st, P.req, (int)S, s->st) != hipSuccess ||
      launch_zero_i32(s->notdone, 1, s->st) != hipSuccess ||
      launch_zero_i32(P.req2, (int)S, s->st) != hipSuccess ||
      hipStreamSynchronize(s->st) != hipSuccess)
    return bail(fail(ctx, SFLS_EDEVICE, "server initialisation failed"));
  uint64_t total = 0;
  total += slot_bytes + (uint64_t)units * s->bpu;
  s->bytes_reserved = total;
  s->stats.units_total = units;
  s->stats.bytes_per_unit = s->bpu;
  s->stats.bytes_reserved = total;
  *out = s;
  return SFLS_OK;
}

sfls_status sfls_server_footprint(const sfls_server* s, int64_t n, uint64_t* bytes) {
  if (!s || !bytes) return SFLS_EINVAL;
  if (n < 2 || n > s->cfg.max_n) return SFLS_EINVAL;
  const int64_t blk = std::max<int64_t>(kUnitMin, (int64_t)1 << ilog2_ceil(n));
  *bytes = (uint64_t)blk * s->bpu;
  return SFLS_OK;
}

sfls_status sfls_server_submit(sfls_server* s, const void* y, int64_t n, uint64_t tag) {
  if (!s) return SFLS_EINVAL;
  sfls_ctx* ctx = s->ctx;
  ctx->err.clear();
  if (!y) return fail(ctx, SFLS_EINVAL, "NULL y");
  if (n < 2) return fail(ctx, SFLS_EINVAL, "n = %lld < 2", (long long)n);
  if (n > s->cfg.max_n)
    return fail(ctx, SFLS_EUNSUPPORTED, "n = %lld exceeds the server's max_n = %lld", (long long)n,
                (long long)s->cfg.max_n);
  {
    const int64_t Lb = (int64_t)1 << (int)std::lround(std::log2(s->prm.L_mult * (double)n));
    if (Lb < 2 * n - 1 || Lb < ((int64_t)1 << ilog2_ceil(n)))
      return fail(ctx, SFLS_EINVAL, "grid L = %lld shorter than 2n-1 for n = %lld", (long long)Lb,
                  (long long)n);
  }
  if (s->free_slots.empty()) return SFLS_EAGAIN;
  (void)hipSetDevice(ctx->device);
  const PlanEntry* pe = nullptr;
  if (s->schur) {
    sfls_status ps = plan_for(s, n, &pe);
    if (ps != SFLS_OK) return ps;
  }
  int order = order_of(std::max<int64_t>(kUnitMin, (int64_t)1 << ilog2_ceil(n)) / kUnitMin);
  InstInfo in;
  SchurLayout lay;
  // the block normally fits at the rounded order; a larger one is tried if not
  int64_t b = -1;
  for (; order <= s->buddy.top; ++order) {
    if (!place(s, n, order, 0, pe, in, lay)) continue;
    b = s->buddy.alloc(order);
    break;
  }
  if (order > s->buddy.top) return fail(ctx, SFLS_EUNSUPPORTED, "request of n = %lld does not fit the pool", (long long)n);
  if (b < 0) return SFLS_EAGAIN;
  place(s, n, order, b, pe, in, lay);
  const int slot = *s->free_slots.begin();
  s->free_slots.erase(s->free_slots.begin());
  in.coff = (int64_t)slot * s->cc;
  s->h_info[slot] = in;
  sep_coef((int)n, s->h_coef[slot]);
  s->h_lay[slot] = lay;
  s->h_koff[slot] = in.koff;
  s->slot_flops[(size_t)slot] = pe ? pe->flops : 8.0 * (double)n * (double)n;
  // The tables stay in the pinned mirrors until the next round's admission
  // kernel copies them (the slot's previous occupant finished rounds ago, and
  // its admission was read long before).  A device signal is copied by the
  // same kernel; a host signal now, through the context's upload stream.
  const size_t ybytes = (size_t)n * s->ysz;
  const size_t ydst = (size_t)in.off * s->ysz;
  bool on_device = false;
  {
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, y) == hipSuccess)
      on_device = at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
    (void)hipGetLastError();  // a host pointer the runtime does not know leaves an error
  }
  if (on_device && (reinterpret_cast<uintptr_t>(y) & 7) != 0) {
    s->buddy.release(b, order);
    s->free_slots.insert(slot);
    return fail(ctx, SFLS_EINVAL, "device signal must be 8-byte aligned");
  }
  if (!on_device) {
    hipError_t e = hipMemcpyAsync(static_cast<char*>(s->ypool) + ydst, y, ybytes,
                                  hipMemcpyHostToDevice, s->up);
    if (e == hipSuccess) e = hipStreamSynchronize(s->up);
    if (e != hipSuccess) {
      s->buddy.release(b, order);
      s->free_slots.insert(slot);
      return fail(ctx, SFLS_EDEVICE, "signal copy failed: %s", hipGetErrorString(e));
    }
  }
  {
    const size_t i = s->admitted.size();
    AdmitRec& r = s->h_adm[(size_t)s->abuf * (size_t)s->cfg.max_slots + i];
    r.slot = slot;
    r.pad_ = 0;
    r.src = on_device ? y : nullptr;
    r.dst_bytes = (int64_t)ydst;
    r.bytes = (int64_t)ybytes;
    s->h_newlist[(size_t)s->abuf * (size_t)s->cfg.max_slots + i] = slot;
  }
  Slot& sl = s->slots[(size_t)slot];
  sl.state = SLOT_ADMITTED;
  sl.order = order;
  sl.block = b;
  sl.tag = tag;
  sl.t_submit = s->now();
  s->hw = std::max(s->hw, slot + 1);
  s->admitted.push_back(slot);
  s->stats.admitted += 1;
  s->stats.in_flight += 1;
  s->stats.units_used += kUnitMin << order;
  return SFLS_OK;
}

sfls_status sfls_server_launch(sfls_server* s) {
  if (!s) return SFLS_EINVAL;
  sfls_ctx* ctx = s->ctx;
  if (s->in_flight) return SFLS_OK;
  if (s->stats.in_flight == 0) return SFLS_OK;
  (void)hipSetDevice(ctx->device);
  const hipStream_t st = s->st;
  const int B = s->hw;
  // newly admitted requests: initial state (phase START) and first step, before this round's evaluation kernels
  const int nnew = (int)s->admitted.size();
  if (nnew > 0) {
    // the kernels read the records and lists from pinned host memory; the
    // buffer flips, so submissions during this round fill the other one, and
    // this one is rewritten only after this round has completed
    const size_t o = (size_t)s->abuf * (size_t)s->cfg.max_slots;
    HIP_TRY(launch_admit(s->m_adm + o, nnew, s->m_info, s->m_coef, s->schur ? s->m_lay : nullptr,
                         s->m_koff, s->dinfo, s->dcoef, s->dlay, s->dkoff, s->ypool, st));
    HIP_TRY(launch_init_state(s->dinfo, s->ypool, s->cfg.ydtype, s->P.st, s->P.req, nnew, st,
                              s->m_newlist + o));
    // their first step (initialisation, the request of the first evaluation
    // and grid sweep) now, so that this round already evaluates them
    HIP_TRY(launch_driver(s->dinfo, s->dprm, s->P, B, st, 2));
    s->abuf ^= 1;
    for (int sl : s->admitted) {
      s->slots[(size_t)sl].state = SLOT_RUNNING;
      // what that step requests (the device overwrites it at the round's end)
      s->h_req[sl] = REQ_EVAL | REQ_GRID | REQ_APPROX;
    }
    s->admitted.clear();
  }
  // sizes of this round's launches, over the requests that asked for work
  int maxN = 0, maxP = 0, lo_n = 1 << 30, hi_n = 0, maxM2 = 0, R2 = 1;
  bool any_eval = false, any_req = false;
  for (int b = 0; b < B; ++b) {
    const int32_t rq = s->h_req[b];
    if (!rq || s->slots[(size_t)b].state != SLOT_RUNNING) continue;
    const InstInfo& in = s->h_info[b];
    any_req = true;
    maxP = std::max(maxP, in.P);
    lo_n = std::min(lo_n, in.N);
    hi_n = std::max(hi_n, in.N);
    // any request may reach the round's grid stage (a sweep it began with,
    // or one its first driver pass asks for)
    maxM2 = std::max(maxM2, in.M);
    R2 = std::max(R2, in.R);
    if (rq & REQ_EVAL) {
      any_eval = true;
      maxN = std::max(maxN, in.N);
    }
  }
  // requests of different sizes: the per-instance kernels whose time grows
  // with N take the slots longest first (slots without work last).  The
  // previous round has completed, so its table is free to rewrite.
  const int32_t* dorder = nullptr;
  if (any_req && lo_n != hi_n) {
    int32_t* o = s->h_order;
    for (int b = 0; b < B; ++b) o[b] = b;
    auto key = [&](int32_t b) {
      return (s->h_req[b] && s->slots[(size_t)b].state == SLOT_RUNNING) ? s->h_info[b].N : 0;
    };
    std::stable_sort(o, o + B, [&](int32_t a, int32_t b) { return key(a) > key(b); });
    dorder = s->m_order;
  }
  DrvPools& P = s->P;
  const int prec = s->prm.precision;
  // per-kernel events and algorithmic work when the context times
  s->timed = ctx->timing != 0;
  s->tmode = ctx->timing;  // the round's events follow the mode at its launch
  if (s->timed && !s->tev[0]) {
    for (auto& e : s->tev) HIP_TRY(hipEventCreate(&e));
  }
  for (int k = 0; k < KID_COUNT; ++k) {
    s->tlaunched[k] = s->tlaunched2[k] = false;
    s->tflops[k] = 0.0;
    s->tbytes[k] = 0.0;
  }
  if (s->timed) {
    const double esz = (double)s->esz, ysz = (double)s->ysz;
    for (int b = 0; b < B; ++b) {
      const int32_t rq = s->h_req[b];
      if (!rq || s->slots[(size_t)b].state != SLOT_RUNNING) continue;
      const InstInfo& in = s->h_info[b];
      const double N = (double)in.N;
      if (rq & REQ_EVAL) {
        s->tflops[KID_FACTOR] += s->slot_flops[(size_t)b];
        s->tbytes[KID_FACTOR] += 40.0 * N;
        if (s->schur) s->tflops[KID_REFINE] += 10.0 * 5.0 * in.P * in.logP + 96.0 * in.P;
        s->tbytes[KID_APPLY] += ysz * N + 32.0 * N;
      }
      if (rq & REQ_GRID) s->tbytes[KID_GRID] += 16.0 * N + 16.0 * (2.0 * N - 1.0) + esz * in.L;
    }
  }
  auto tstart = [&](int k) -> hipError_t {
    s->tlaunched[k] = true;
    return s->timed && times_kernel(s->tmode, k) ? hipEventRecord(s->tev[2 * k], st) : hipSuccess;
  };
  auto tstop = [&](int k) -> hipError_t {
    return s->timed && times_kernel(s->tmode, k) ? hipEventRecord(s->tev[2 * k + 1], st) : hipSuccess;
  };
  const int E2 = 2 * KID_COUNT;
  auto tstart2 = [&](int k) -> hipError_t {
    s->tlaunched2[k] = true;
    return s->timed && times_kernel(s->tmode, k) ? hipEventRecord(s->tev[E2 + 2 * k], st)
                                            : hipSuccess;
  };
  auto tstop2 = [&](int k) -> hipError_t {
    return s->timed && times_kernel(s->tmode, k) ? hipEventRecord(s->tev[E2 + 2 * k + 1], st)
                                            : hipSuccess;
  };
  if (any_eval) {
    HIP_TRY(tstart(KID_GEN));
    HIP_TRY(launch_toeplitz_column(s->dinfo, P.req, P.K_e, P.th_e, P.ga_e, P.beta_e, s->c, B, maxN,
                                   st, ctx->nufft_mode, ctx->tws64, s->scratch, maxP));
    HIP_TRY(tstop(KID_GEN));
    HIP_TRY(tstart(KID_FACTOR));
    if (s->schur) {
      HIP_TRY(launch_schur(s->dinfo, P.req, s->dlay, s->dacts, s->c, ctx->tw64, ctx->logtw,
                           ctx->tws64, s->sscr, s->rho, s->delta, s->logdet, s->lev_status,
                           s->failed, B, s->Fmax, st, dorder));
    } else {
      HIP_TRY(launch_levinson(s->dinfo, P.req, s->c, s->rho, s->delta, s->logdet, s->lev_status,
                              s->failed, B, (int)s->cfg.max_n, st));
    }
    HIP_TRY(tstop(KID_FACTOR));
    HIP_TRY(tstart(KID_REFINE));
    if (s->schur)
      HIP_TRY(launch_gen_refine(s->dinfo, P.req, s->lev_status, s->c, s->rho, s->delta, ctx->tw64,
                                ctx->logtw, ctx->tws64, s->scratch, s->rf_r, s->rf_dx, B, maxP, st,
                                dorder));
    HIP_TRY(launch_logdet_lemma(s->dinfo, P.req, P.K_e, P.th_e, P.ga_e, P.beta_e, s->lev_status,
                                s->logdet, B, st));
    HIP_TRY(tstop(KID_REFINE));
    HIP_TRY(tstart(KID_APPLY));
    HIP_TRY(launch_gs_apply(s->dinfo, P.req, s->ypool, s->cfg.ydtype, s->rho, s->delta, ctx->tw64,
                            ctx->logtw, ctx->tws64, s->scratch, s->w, s->yCy, s->ww, B, maxP, st,
                            dorder));
    HIP_TRY(tstop(KID_APPLY));
  }
  // active-set vectors at the evaluated points (candidates follow the grid stage)
  if (any_eval) {
    HIP_TRY(tstart(KID_ACTIVE));
    HIP_TRY(launch_active(s->dinfo, P.req, P.K_e, nullptr, s->prefix, B, P.th_e, s->cand, s->w,
                          s->rho, s->delta, s->dcoef, s->evq, s->evr, s->evu, s->evs, s->evt,
                          s->evv, s->evx, s->cq, s->cs, 2048, ctx->nufft_mode, ctx->tws64,
                          s->scratch, maxP, st));
    HIP_TRY(tstop(KID_ACTIVE));
  }
  // first driver pass: the slots whose request had no grid sweep
  HIP_TRY(tstart(KID_DRIVER));
  HIP_TRY(launch_driver(s->dinfo, s->dprm, P, B, st));  // request bits also to h_req
  HIP_TRY(tstop(KID_DRIVER));
  if (any_req) {
    // grid stage, after the first pass: the sweeps the round began with and
    // those the pass just requested at the point this round evaluated (run
    // now instead of a round later); then candidates and the second pass,
    // for exactly these slots (P.req2)
    const void* tw = prec == SFLS_FP64 ? (const void*)ctx->tws64 : (const void*)ctx->tws32;
    const double slack = prec == SFLS_FP64 ? 1e-9 : 1e-3;
    HIP_TRY(tstart2(KID_OMEGA));
    HIP_TRY(launch_omega(s->dinfo, P.req2, s->rho, s->delta, s->dcoef, ctx->tws64, s->scratch, 1,
                         1, s->oms, nullptr, nullptr, nullptr, nullptr, B, maxP, st, dorder));
    HIP_TRY(tstop2(KID_OMEGA));
    HIP_TRY(tstart2(KID_GRID));
    HIP_TRY(launch_grid(prec, s->dinfo, P.req2, s->w, s->oms, P.gbar_e, P.zeta_e, tw, ctx->logtw,
                        R2, B, maxM2, nullptr, nullptr, s->dL, s->pv, s->pi, st));
    HIP_TRY(tstop2(KID_GRID));
    HIP_TRY(tstart2(KID_SELECT));
    HIP_TRY(launch_select(prec, s->dinfo, P.req2, s->dL, R2, s->pv, s->pi, s->prm.approx_ratio,
                          slack, s->prm.cand_cap, s->cand, s->ncand, s->ovf, B, st));
    HIP_TRY(tstop2(KID_SELECT));
    HIP_TRY(tstart2(KID_ACTIVE));
    HIP_TRY(launch_active(s->dinfo, P.req2, P.K_e, s->ncand, s->prefix, B, P.th_e, s->cand, s->w,
                          s->rho, s->delta, s->dcoef, s->evq, s->evr, s->evu, s->evs, s->evt,
                          s->evv, s->evx, s->cq, s->cs, 2048, ctx->nufft_mode, ctx->tws64,
                          s->scratch, maxP, st));
    HIP_TRY(tstop2(KID_ACTIVE));
    HIP_TRY(tstart2(KID_DRIVER));
    HIP_TRY(launch_driver(s->dinfo, s->dprm, P, B, st, 1));
    HIP_TRY(tstop2(KID_DRIVER));
  }
  HIP_TRY(hipEventRecord(s->ev, st));
  s->in_flight = true;
  s->t_launch = std::chrono::steady_clock::now();
  return SFLS_OK;
}

sfls_status sfls_server_wait(sfls_server* s, int32_t block, int32_t* ready, int32_t* finished) {
  if (!s) return SFLS_EINVAL;
  sfls_ctx* ctx = s->ctx;
  if (finished) *finished = 0;
  if (ready) *ready = 1;
  if (!s->in_flight) return SFLS_OK;
  (void)hipSetDevice(ctx->device);
  if (!block) {
    const hipError_t q = hipEventQuery(s->ev);
    if (q == hipErrorNotReady) {
      if (ready) *ready = 0;
      return SFLS_OK;
    }
    if (q != hipSuccess) return fail(ctx, SFLS_EDEVICE, "round failed: %s", hipGetErrorString(q));
  } else {
    HIP_TRY(spin_wait(s->ev));
  }
  s->in_flight = false;
  s->stats.rounds += 1;
  // grid sweeps of the second stage: their traffic (entries are cleared
  // once read; the device writes them in its next first pass)
  for (int b = 0; b < s->hw; ++b) {
    if (!s->h_req2[b]) continue;
    s->h_req2[b] = 0;
    const double N = (double)s->h_info[b].N;
    s->tbytes[KID_GRID] += 16.0 * N + 16.0 * (2.0 * N - 1.0) + (double)s->esz * s->h_info[b].L;
  }
  if (s->timed) {
    const int E2 = 2 * KID_COUNT;
    for (int k = 0; k < KID_COUNT; ++k) {
      if (!times_kernel(s->tmode, k)) continue;
      for (int sg = 0; sg < 2; ++sg) {
        if (!(sg ? s->tlaunched2[k] : s->tlaunched[k])) continue;
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, s->tev[sg * E2 + 2 * k], s->tev[sg * E2 + 2 * k + 1]));
        ctx->kst[k].launches += 1;
        ctx->kst[k].seconds += 1e-3 * (double)ms;
      }
      ctx->kst[k].flops += s->tflops[k];
      ctx->kst[k].bytes += s->tbytes[k];
    }
  }
  s->stats.gpu_seconds +=
      std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t_launch).count();
  const double t_done = s->now();
  // results gathered behind the previous round are complete by now
  sfls_status fs = finish_gather(s);
  if (fs != SFLS_OK) return fs;
  // requests whose driver asked for nothing more have finished: release their
  // slots and blocks, and pack their outputs behind this round
  int nf = 0;
  int64_t ctot = 0;
  for (int b = 0; b < s->hw; ++b) {
    if (s->slots[(size_t)b].state != SLOT_RUNNING || s->h_req[b] != 0) continue;
    s->h_list[nf] = b;
    s->h_doff[nf] = ctot;
    s->h_gkoff[nf] = s->h_info[b].koff;
    ctot += 4 * (int64_t)s->h_info[b].kcap;
    ++nf;
  }
  if (nf == 0) return SFLS_OK;
  if ((size_t)ctot > s->h_comp_n) {
    size_t want = std::max<size_t>((size_t)ctot, 2 * s->h_comp_n);
    auto it = std::find(s->host_owned.begin(), s->host_owned.end(), (void*)s->h_comp);
    if (it != s->host_owned.end()) s->host_owned.erase(it);
    if (s->h_comp) (void)hipHostFree(s->h_comp);
    s->h_comp = nullptr;
    s->h_comp_n = 0;
    if (halloc(&s->h_comp, want, s->host_owned) != hipSuccess)
      return fail(ctx, SFLS_ENOMEM, "pinned result staging of %zu doubles", want);
    HIP_TRY(hipHostGetDevicePointer((void**)&s->m_comp, s->h_comp, 0));
    s->h_comp_n = want;
  }
  const hipStream_t st = s->st;
  const DrvPools& P = s->P;
  // the gather reads its lists from, and writes the packed results into,
  // pinned host memory (no copies); the host touches them again only after
  // ev_res
  HIP_TRY(launch_gather_results(s->m_list, s->m_doff, nf, s->m_gkoff, P.out_K, P.out_theta,
                                P.out_alpha, P.out_gamma, P.out_beta, P.out_zeta, P.out_obj,
                                P.out_iters, P.out_evals, P.out_status, s->m_res, s->m_comp, st));
  HIP_TRY(hipEventRecord(s->ev_res, st));
  s->gathering.clear();
  for (int i = 0; i < nf; ++i) {
    const int b = s->h_list[i];
    Slot& sl = s->slots[(size_t)b];
    Result out;
    out.r.tag = sl.tag;
    out.r.n = s->h_info[b].N;
    out.r.t_submit = sl.t_submit;
    out.r.t_done = t_done;
    s->gathering.push_back(std::move(out));
    // the slot and its block can take a new request now: every later write
    // to them is ordered after the gather on this stream, and the gather
    // reads no table a new admission rewrites
    s->buddy.release(sl.block, sl.order);
    s->stats.units_used -= kUnitMin << sl.order;
    sl = Slot{};
    s->free_slots.insert(b);
  }
  s->gather_pending = true;
  while (s->hw > 0 && s->slots[(size_t)s->hw - 1].state == SLOT_FREE) --s->hw;
  s->stats.completed += nf;
  s->stats.in_flight -= nf;
  if (finished) *finished = nf;
  return SFLS_OK;
}

sfls_status sfls_server_step(sfls_server* s, int32_t* finished) {
  sfls_status r = sfls_server_launch(s);
  if (r != SFLS_OK) return r;
  int32_t ready = 0;
  return sfls_server_wait(s, 1, &ready, finished);
}

sfls_status sfls_server_poll(sfls_server* s, sfls_result* res, int32_t max_results,
                             double* theta, double* gamma, double* alpha, int64_t comp_cap,
                             int32_t* nres) {
  if (!s || !nres || (max_results > 0 && !res)) return SFLS_EINVAL;
  *nres = 0;
  (void)hipSetDevice(s->ctx->device);
  sfls_status fs = finish_gather(s);
  if (fs != SFLS_OK) return fs;
  int64_t used = 0;
  while (*nres < max_results && !s->done.empty()) {
    Result& r = s->done.front();
    const int64_t K = r.r.K;
    if (K > 0 && (!theta || !gamma || !alpha || used + K > comp_cap)) {
      if (*nres == 0)
        return fail(s->ctx, SFLS_EINVAL, "comp_cap = %lld too small for a result of K = %lld",
                    (long long)comp_cap, (long long)K);
      break;
    }
    sfls_result o = r.r;
    o.comp_off = used;
    if (K > 0) {
      std::memcpy(theta + used, r.comp.data(), (size_t)K * sizeof(double));
      std::memcpy(gamma + used, r.comp.data() + K, (size_t)K * sizeof(double));
      std::memcpy(alpha + 2 * used, r.comp.data() + 2 * K, (size_t)(2 * K) * sizeof(double));
    }
    used += K;
    res[(*nres)++] = o;
    s->done.pop_front();
  }
  return SFLS_OK;
}

sfls_status sfls_server_get_stats(const sfls_server* s, sfls_server_stats* out) {
  if (!s || !out) return SFLS_EINVAL;
  *out = s->stats;
  return SFLS_OK;
}

}  // extern "C"
