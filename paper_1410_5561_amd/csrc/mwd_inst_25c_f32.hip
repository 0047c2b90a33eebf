// MWD instantiations for the 25c stencil in f32.
#include "mwd_rows.hpp"

namespace mwd {

static const MwdEntry kEntries[] = {
    MWD_ENTRY(K25C, float, 1, 8, 1), MWD_ENTRY(K25C, float, 1, 16, 1), MWD_ENTRY(K25C, float, 1, 8, 2),
};

void mwd_table_25c_f32(const MwdEntry** tab, int* n)
{
    *tab = kEntries;
    *n = (int)(sizeof(kEntries) / sizeof(kEntries[0]));
}

}  // namespace mwd
