// sfls_gs_apply_noalloc: sfls_gs_apply for callers that cannot allocate device
// memory.  The per-call device memory beyond the caller's buffers (the
// instance table and the convolution scratch of the apply) comes from one
// static device array of fixed size, held by every device the library runs
// on until the process ends.
#include <mutex>

#include "host_internal.hpp"
#include "k_launch.hpp"
#include "sfls.h"

using namespace sfls;
using namespace sfls_host;

static __device__ __align__(256) unsigned char scratch[SFLS_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_mu;
void* g_scratch[NOALLOC_MAX_DEVICES] = {};  // device address of `scratch` per device
}  // namespace

namespace sfls_host {

// Device address of this device's copy of `scratch`.  Called by sfls_create
// with the context's device current; the address is looked up once per device
// and kept.  The array's name is a host-side stand-in: host code uses only the
// looked-up address.
sfls_status noalloc_init(sfls_ctx* ctx) {
  if (ctx->device < 0 || ctx->device >= NOALLOC_MAX_DEVICES)
    return fail(ctx, SFLS_EUNSUPPORTED, "device %d: no scratch slot", ctx->device);
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[ctx->device]) return SFLS_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(ctx, SFLS_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
  g_scratch[ctx->device] = p;
  return SFLS_OK;
}

}  // namespace sfls_host

extern "C" sfls_status sfls_gs_apply_noalloc(sfls_ctx* ctx, int64_t B, const int64_t* n,
                                             const int64_t* off, const void* y, int32_t ydtype,
                                             const double* rho, const double* delta, double* w,
                                             double* yCy, double* ww, void* stream) {
  if (!ctx) return SFLS_EINVAL;
  ctx->err.clear();
  sfls_status s = check_batch(ctx, B, n, off, 1);
  if (s != SFLS_OK || B == 0) return s;
  if (!y || !rho || !delta || !w) return fail(ctx, SFLS_EINVAL, "NULL argument");
  if (ydtype != SFLS_C64 && ydtype != SFLS_C128) return fail(ctx, SFLS_EINVAL, "bad ydtype");
  Sizes sz;
  int64_t pt = 0;
  std::vector<InstInfo> info = base_info(B, n, off, sz, pt);
  const size_t info_bytes = ((size_t)B * sizeof(InstInfo) + 255) & ~(size_t)255;
  const size_t need = info_bytes + (size_t)pt * sizeof(cd);
  if (need > (size_t)SFLS_NOALLOC_SCRATCH_BYTES)
    return fail(ctx, SFLS_EUNSUPPORTED,
                "batch needs %zu bytes of scratch; sfls_gs_apply_noalloc has %zu", need,
                (size_t)SFLS_NOALLOC_SCRATCH_BYTES);
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    base = g_scratch[ctx->device];
  }
  if (!base) return fail(ctx, SFLS_EDEVICE, "scratch of device %d not set up", ctx->device);
  (void)hipSetDevice(ctx->device);
  hipStream_t st = as_stream(stream);
  InstInfo* dinfo = static_cast<InstInfo*>(base);
  cd* scr = reinterpret_cast<cd*>(static_cast<unsigned char*>(base) + info_bytes);
  // the table is copied from host memory before the kernel reads it (the copy
  // is ordered on the stream; the wait keeps `info` alive until it is done)
  HIP_TRY(hipMemcpyAsync(dinfo, info.data(), (size_t)B * sizeof(InstInfo), hipMemcpyHostToDevice, st));
  HIP_TRY(launch_gs_apply(dinfo, nullptr, y, ydtype, (const cd*)rho, delta, ctx->tw64, ctx->logtw,
                          ctx->tws64, scr, (cd*)w, yCy, ww, (int)B, sz.maxP, st));
  HIP_TRY(hipStreamSynchronize(st));
  return SFLS_OK;
}
