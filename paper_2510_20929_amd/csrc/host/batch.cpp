// Batched uneven reconstructions (placeholder until the persistent batched kernel lands).
#include <hip/hip_runtime.h>

#include "../../../include/ptyhip.h"

extern "C" {
ptyhip_status ptyhip_batch_create(const ptyhip_desc*, const int32_t*, int32_t, const ptyhip_tune*, ptyhip_batch* out) {
  if (out) *out = nullptr;
  return PTYHIP_EUNSUPPORTED;
}
ptyhip_status ptyhip_batch_bind(ptyhip_batch, int32_t, const float*, const float*, const float*, const float*,
                                const float*, double*, float*, float*, float*, float*) {
  return PTYHIP_EUNSUPPORTED;
}
ptyhip_status ptyhip_batch_launch(ptyhip_batch, void*, uint32_t) { return PTYHIP_EUNSUPPORTED; }
ptyhip_status ptyhip_batch_get_error(ptyhip_batch, void*, uint32_t*) { return PTYHIP_EUNSUPPORTED; }
void ptyhip_batch_destroy(ptyhip_batch) {}
}
