// Entry points declared in include/dsnlm.h that this build does not provide yet.
#include "internal.h"

using namespace dsnlm;

extern "C" {

int dsnlm_apply_backward(const dsnlm_weights*, const float*, const float*, float*, float*, float*,
                         void*) {
    return fail(DSNLM_EUNSUPPORTED, "dsnlm_apply_backward: not available in this build");
}

int ladmm_step(const ladmm_operator*, const ladmm_params*, int, dsnlm_weights**, float*, float*,
               float*, void*) {
    return fail(DSNLM_EUNSUPPORTED, "ladmm_step: not available in this build");
}

int ladmm_solve(const ladmm_operator*, const ladmm_params*, float*, float*, float*, float*, float*,
                void*) {
    return fail(DSNLM_EUNSUPPORTED, "ladmm_solve: not available in this build");
}

int ladmm_apply_forward(const ladmm_operator*, const float*, float*, void*) {
    return fail(DSNLM_EUNSUPPORTED, "ladmm_apply_forward: not available in this build");
}

int ladmm_gradient(const ladmm_operator*, const float*, float*, void*) {
    return fail(DSNLM_EUNSUPPORTED, "ladmm_gradient: not available in this build");
}

int ladmm_operator_norm2(const ladmm_operator*, int, float*, void*) {
    return fail(DSNLM_EUNSUPPORTED, "ladmm_operator_norm2: not available in this build");
}

}  // extern "C"
