// Learned weight proposer (placeholder until the MLP kernels land).
#include "common.h"

namespace morap {
struct Proposer {};
void proposer_destroy(Proposer* p) { delete p; }
bool proposer_ready(const morap_ctx*, int, int) { return false; }
void proposer_infer_host(morap_ctx*, const float*, int, float*) {
    fail(MORAP_E_UNSUPPORTED, "proposer not built");
}
}  // namespace morap

extern "C" {
int morap_proposer_init(morap_ctx*, int, int, uint64_t) { return MORAP_E_UNSUPPORTED; }
int64_t morap_proposer_num_params(const morap_ctx*) { return 0; }
int morap_proposer_get_params(const morap_ctx*, float*) { return MORAP_E_UNSUPPORTED; }
int morap_proposer_set_params(morap_ctx*, const float*) { return MORAP_E_UNSUPPORTED; }
int morap_proposer_infer(morap_ctx*, const float*, int, float*) { return MORAP_E_UNSUPPORTED; }
int morap_proposer_step(morap_ctx*, const float*, const float*, int, const morap_train_opts*, int, float*,
                        float*) {
    return MORAP_E_UNSUPPORTED;
}
int morap_proposer_train(morap_ctx*, const float*, const float*, int, const morap_train_opts*, float*) {
    return MORAP_E_UNSUPPORTED;
}
int morap_proposer_save(const morap_ctx*, const char*) { return MORAP_E_UNSUPPORTED; }
int morap_proposer_load(morap_ctx*, const char*) { return MORAP_E_UNSUPPORTED; }
}
