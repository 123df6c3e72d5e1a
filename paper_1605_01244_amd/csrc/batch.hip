// Batched evaluation of several plans.  (Persistent single-launch scheduler
// is added on top of the per-stage kernels; this file owns its dispatch.)
#include "internal.h"

namespace nfft3 {

int launch_batch(int T, nfft3_plan_impl *const *plans, const void *const *fhat, void *const *out,
                 int deriv_mask) {
    for (int t = 0; t < T; ++t) {
        nfft3_plan_impl *p = plans[t];
        hipStream_t saved = p->stream;
        p->stream = plans[0]->stream;
        char *o = (char *)out[t];
        int rc = NFFT3_OK;
        for (int field = -1; field < 3 && rc == NFFT3_OK; ++field) {
            if (field >= 0 && !(deriv_mask & (1 << field))) continue;
            rc = launch_grid_forward(p, fhat[t], p->grid, field);
            if (rc == NFFT3_OK) rc = launch_interp(p, p->grid, o);
            o += (size_t)p->M * p->elt;
        }
        p->stream = saved;
        if (rc) return rc;
    }
    return NFFT3_OK;
}

}  // namespace nfft3

namespace nfft3 {
int64_t g_spin_limit = INT64_MAX;
}

extern "C" int nfft3_batch_set_spin_limit(int64_t spins) {
    nfft3::g_spin_limit = spins <= 0 ? INT64_MAX : spins;
    return NFFT3_OK;
}
