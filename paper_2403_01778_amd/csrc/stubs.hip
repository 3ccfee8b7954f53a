// Entry points whose implementation lands in later files of this library.
#include "common.h"
#include "tuning.h"

extern "C" {

size_t hoscf_extra_workspace_size(int op, const hoscf_tensor* T) {
    (void)op;
    (void)T;
    return 0;
}

int hoscf_backward(const hoscf_tensor*, const double*, double, double, const double*, void*, int, double*, double*,
                   void*, size_t, void*) {
    return HOSCF_INVALID_ARG;
}

int hoscf_ttvc_backward(const hoscf_tensor*, const double*, const void*, const double*, const double*, double, void*,
                        int, double*, void*, size_t, void*) {
    return HOSCF_INVALID_ARG;
}

int hoscf_batch_plan_create(int, const hoscf_tensor*, int, const hoscf_options*, hoscf_plan** out) {
    if (out) *out = nullptr;
    return HOSCF_INVALID_ARG;
}
void hoscf_plan_destroy(hoscf_plan*) {}
size_t hoscf_batch_workspace_size(const hoscf_plan*) { return 0; }
int hoscf_solve_batched(const hoscf_plan*, const double*, double*, double*, int32_t*, int32_t*, void*, size_t, void*) {
    return HOSCF_INVALID_ARG;
}

}
