// Adaptive direction sets (Section 2.1.3, Fig. 1).
#include "rt_internal.h"

using namespace rt;

extern "C" rt_status rt_dirset_adaptive(const rt_model* model, int32_t lmin, int32_t lmax,
                                        const int32_t* sample_ids_dev, int64_t n_sample,
                                        const int32_t* origins_dev, int64_t n_origins, void* stream,
                                        rt_dirset** out) {
    (void)model; (void)lmin; (void)lmax; (void)sample_ids_dev; (void)n_sample; (void)origins_dev;
    (void)n_origins; (void)stream;
    if (out) *out = nullptr;
    return fail(RT_ERR_UNSUPPORTED, "rt_dirset_adaptive: not available in this build");
}
