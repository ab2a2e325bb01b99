// Reverse-mode (adjoint) products of the FR/CPR residual: placeholder until the
// gather-formulated adjoint kernels are in.
#include "fr_internal.hpp"

fr_status launch_vjp(fr_ctx c, const double* q, const double* w, double* out, hipStream_t s) {
    (void)c; (void)q; (void)w; (void)out; (void)s;
    fr_set_error("fr_vjp: not built yet");
    return FR_EUNSUPPORTED;
}
