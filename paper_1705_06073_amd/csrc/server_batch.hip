// Batched admission: several requests in one call, for hosts whose per-call
// overhead (a Python binding's, say) would otherwise sit between two rounds.
#include <hip/hip_runtime.h>

#include "sfls.h"

extern "C" sfls_status sfls_server_submit_many(sfls_server* srv, int32_t count,
                                               const void* const* ys, const int64_t* ns,
                                               const uint64_t* tags, int32_t* accepted) {
  if (accepted) *accepted = 0;
  if (!srv || count < 0 || !accepted || (count > 0 && (!ys || !ns || !tags)))
    return SFLS_EINVAL;
  for (int32_t i = 0; i < count; ++i) {
    const sfls_status s = sfls_server_submit(srv, ys[i], ns[i], tags[i]);
    if (s == SFLS_EAGAIN) return SFLS_OK;
    if (s != SFLS_OK) return s;
    *accepted = i + 1;
  }
  return SFLS_OK;
}
