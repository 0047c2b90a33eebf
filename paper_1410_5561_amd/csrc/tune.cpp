#include "tune.hpp"

#include "../../include/mwd_stencil.h"

namespace mwd {

MwdShape default_shape(int kind, int dtype)
{
    if (kind == K25C || kind == K25V) return MwdShape{16, 1};
    if (kind == K7V && dtype == 0) return MwdShape{8, 1};
    return MwdShape{8, 2};
}

int tune_choose(int kind, int dtype, int nx, int ny, int nz, TuneChoice* out)
{
    (void)nx; (void)ny; (void)nz;
    out->mode = STENCIL_MODE_MWD;
    out->shape = default_shape(kind, dtype);
    return STENCIL_OK;
}

MwdShape tune_batch_shape(int kind, int dtype, int nx, int ny, int nz, int T)
{
    (void)dtype; (void)nx; (void)ny; (void)nz; (void)T;
    if (kind == K25C || kind == K25V) return MwdShape{16, 1};
    if (kind == K7V) return MwdShape{4, 4};
    return MwdShape{8, 2};
}

}  // namespace mwd
