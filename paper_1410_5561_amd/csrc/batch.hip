#include "batch.hpp"
#include "internal.hpp"

namespace mwd {

struct BatchState {
    int dummy;
};

int batch_run(int, int, BatchState**, stencil_grid*, const stencil_coeffs*, int, int, hipStream_t)
{
    set_last_error("batched runs are not built yet");
    return STENCIL_EUNSUPPORTED;
}

void batch_free(BatchState* s) { delete s; }

}  // namespace mwd
