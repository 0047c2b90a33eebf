// MWD instantiations for the 7c stencil in f32.
#include "mwd_rows.hpp"

namespace mwd {

static const MwdEntry kEntries[] = {
    MWD_ENTRY(K7C, float, 1, 4, 1), MWD_ENTRY(K7C, float, 1, 4, 2), MWD_ENTRY(K7C, float, 1, 8, 1),
    MWD_ENTRY(K7C, float, 1, 8, 2), MWD_ENTRY(K7C, float, 1, 16, 1), MWD_ENTRY(K7C, float, 1, 4, 4),
};

void mwd_table_7c_f32(const MwdEntry** tab, int* n)
{
    *tab = kEntries;
    *n = (int)(sizeof(kEntries) / sizeof(kEntries[0]));
}

}  // namespace mwd
