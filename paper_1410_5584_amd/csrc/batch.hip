// Batched replicas (not built yet): every entry point reports FMLB_E_UNSUPPORTED.
#include <hip/hip_runtime.h>

#include "../../include/fmlb.h"

struct fmlb_batch {
    int unused;
};

extern "C" {
size_t fmlb_batch_required_bytes(const fmlb_params *, int, int) { return 0; }
fmlb_status fmlb_batch_create(const fmlb_params *, int, void *, void *const[3], fmlb_batch **out)
{
    if (out) *out = nullptr;
    return FMLB_E_UNSUPPORTED;
}
void fmlb_batch_destroy(fmlb_batch *b) { delete b; }
fmlb_status fmlb_batch_init_density(fmlb_batch *, int, const double *, const double *) { return FMLB_E_UNSUPPORTED; }
fmlb_status fmlb_batch_step(fmlb_batch *, int64_t, int) { return FMLB_E_UNSUPPORTED; }
fmlb_status fmlb_batch_get_populations(fmlb_batch *, int, double *, size_t) { return FMLB_E_UNSUPPORTED; }
fmlb_status fmlb_batch_global_sums(fmlb_batch *, int, double *) { return FMLB_E_UNSUPPORTED; }
fmlb_status fmlb_batch_mode_accumulate(fmlb_batch *) { return FMLB_E_UNSUPPORTED; }
fmlb_status fmlb_batch_mode_variances(fmlb_batch *, int, double *, int64_t *) { return FMLB_E_UNSUPPORTED; }
fmlb_status fmlb_batch_set_tile(fmlb_batch *, int, int) { return FMLB_E_UNSUPPORTED; }
int64_t fmlb_batch_total_sites(const fmlb_batch *) { return -1; }
}
