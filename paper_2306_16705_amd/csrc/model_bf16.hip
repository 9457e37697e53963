// BF16 MFMA forward of the amplitude transformer and the phase MLP.
#include "model.hpp"

namespace nnqs {

nnqs_status bf16_model_init(nnqs_model *m, const float *weights) {
    (void)weights;
    m->bf16_ok = false;
    return NNQS_OK;
}

void bf16_model_free(nnqs_model *m) {
    hipFree(m->d_bf16);
    hipFree(m->d_f32);
    m->d_bf16 = nullptr;
    m->d_f32 = nullptr;
}

nnqs_status enqueue_logpsi_bf16(const nnqs_model *m, const uint64_t *keys, int64_t n, double *logabs, double *phase,
                                hipStream_t st) {
    (void)m; (void)keys; (void)n; (void)logabs; (void)phase; (void)st;
    return fail(NNQS_EUNSUPPORTED, "BF16 forward not available for this model");
}

}  // namespace nnqs
