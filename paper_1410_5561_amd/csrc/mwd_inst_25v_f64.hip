// MWD instantiations for the 25v stencil in f64.
#include "mwd_rows.hpp"

namespace mwd {

static const MwdEntry kEntries[] = {
    MWD_ENTRY(K25V, double, 0, 8, 1), MWD_ENTRY(K25V, double, 0, 16, 1), MWD_ENTRY(K25V, double, 0, 8, 2),
};

void mwd_table_25v_f64(const MwdEntry** tab, int* n)
{
    *tab = kEntries;
    *n = (int)(sizeof(kEntries) / sizeof(kEntries[0]));
}

}  // namespace mwd
