// Adjoint (transpose) of the stage and of the outer step.
#include "../../include/dycore.h"
#include "dycore_internal.h"

struct dycore_s;
size_t dyc_adjoint_workspace_bytes(const dycore_s* h) { (void)h; return 256; }

extern "C" {
int dycore_step_adjoint(dycore_t h, const void*, const void*, const void*, const void*, void*, void*, void*, void*,
                        void*) {
  return h ? DYCORE_EUNSUPPORTED : DYCORE_EINVAL;
}
int dycore_stage_adjoint(dycore_t h, int, double, const void*, const void*, const void*, const void*, const void*,
                         const void*, const void*, const void*, void*, void*, void*, void*, void*, void*, void*,
                         void*, void*) {
  return h ? DYCORE_EUNSUPPORTED : DYCORE_EINVAL;
}
}
