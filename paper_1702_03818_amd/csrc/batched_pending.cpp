#include "internal.h"
using namespace frkc2;
extern "C" size_t frkc2_batched_workspace_bytes(int, const frkc2_grid *, const int *) { return 0; }
extern "C" int frkc2_step_batched(int, const frkc2_grid *, double *const *, const double *const *,
                                  const double *, const int *, double, void *, size_t, hipStream_t)
{ set_error("batched: pending"); return FRKC2_EINVAL; }
extern "C" int frkc2_batched_status(void *, hipStream_t) { return FRKC2_EINVAL; }
