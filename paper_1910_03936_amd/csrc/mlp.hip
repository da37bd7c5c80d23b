// Cost model kernels (placeholder until the model lands).
#include "paf_internal.h"

extern "C" {
paf_status paf_features(paf_ctx*, const paf_batch*, float*, void*) { return PAF_ERR_STATE; }
paf_status paf_mlp_set_params(paf_ctx*, const float*) { return PAF_ERR_STATE; }
paf_status paf_mlp_get_params(paf_ctx*, float*) { return PAF_ERR_STATE; }
paf_status paf_mlp_forward(paf_ctx*, const float*, uint64_t, float*, void*) { return PAF_ERR_STATE; }
paf_status paf_mlp_train_step(paf_ctx*, const float*, const float*, uint64_t, float, float*, float*, void*) { return PAF_ERR_STATE; }
paf_status paf_bucket(paf_ctx*, const paf_batch*, const float*, uint32_t*, uint32_t*, void*) { return PAF_ERR_STATE; }
paf_status paf_filter_bucketed(paf_ctx*, const paf_batch*, uint32_t, const paf_out*, void*) { return PAF_ERR_STATE; }
}
