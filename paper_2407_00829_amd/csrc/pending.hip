// Entry points whose GPU implementations live in later translation units of this library.
#include "plan.h"

extern "C" {
sable_status sable_features(const sable_csr*, void*, float*) { return SABLE_ERR_INTERNAL; }
sable_status sable_class_plan(int32_t, sable_extractor*, int32_t*, sable_thresholds*) { return SABLE_ERR_INTERNAL; }
sable_status sable_mlp_forward(const float*, const float*, int32_t, float*, void*) { return SABLE_ERR_INTERNAL; }
sable_status sable_mlp_train_step(float*, float*, float*, float*, const float*, const int32_t*, int32_t, float, float, float, float, int32_t, void*, float*) { return SABLE_ERR_INTERNAL; }
sable_status sable_batch_create(const sable_plan_t*, const sable_batch_item*, int32_t, void*, sable_batch_t*) { return SABLE_ERR_INTERNAL; }
sable_status sable_batch_run(sable_batch_t, void*) { return SABLE_ERR_INTERNAL; }
sable_status sable_batch_latencies(sable_batch_t, uint64_t*, double*) { return SABLE_ERR_INTERNAL; }
sable_status sable_batch_destroy(sable_batch_t) { return SABLE_ERR_INTERNAL; }
}
