// Batched design variants (declared in include/etm.h).
#include <hip/hip_runtime.h>

#include <string>

#include "etm_internal.h"

struct etm_batch {
  int32_t max_slots = 0;
};

extern "C" {

etm_status etm_batch_create(int32_t max_slots, const char *, etm_batch **out) {
  if (!out || max_slots < 1) return ETM_E_INVAL;
  *out = new etm_batch();
  (*out)->max_slots = max_slots;
  return ETM_OK;
}
etm_status etm_batch_attach(etm_batch *, etm_plan *, int32_t *) { return ETM_E_STATE; }
etm_status etm_batch_detach(etm_batch *, int32_t) { return ETM_E_STATE; }
etm_status etm_batch_advance(etm_batch *, int64_t, void *) { return ETM_E_STATE; }
void etm_batch_destroy(etm_batch *b) { delete b; }

}  // extern "C"
