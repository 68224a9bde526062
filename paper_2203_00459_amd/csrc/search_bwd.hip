// Adjoint of the decoupled search (placeholder until the backward kernels land).
#include "internal.hpp"

namespace fmbym {

size_t bwd_workspace(const fmbym_params& p, int batch) { return fwd_layout(p, batch).total; }

int launch_backward(const Plan&, int, const float*, const float*, const float*, const float*,
                    const float*, const float*, const float*, const float*, const float*, float*,
                    float*, float*, float*, char*, hipStream_t) {
    return FMBYM_EUNSUPPORTED;
}

}  // namespace fmbym
