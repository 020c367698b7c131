// Entry points declared in include/dsnlm.h that this build does not provide yet.
#include "internal.h"

using namespace dsnlm;

extern "C" {

int dsnlm_apply_backward(const dsnlm_weights*, const float*, const float*, float*, float*, float*,
                         void*) {
    return fail(DSNLM_EUNSUPPORTED, "dsnlm_apply_backward: not available in this build");
}

}  // extern "C"
