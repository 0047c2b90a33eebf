// MWD instantiations for the 7v stencil in f32.
#include "mwd_rows.hpp"

namespace mwd {

static const MwdEntry kEntries[] = {
    MWD_ENTRY(K7V, float, 1, 4, 1), MWD_ENTRY(K7V, float, 1, 4, 2), MWD_ENTRY(K7V, float, 1, 8, 1),
    MWD_ENTRY(K7V, float, 1, 8, 2), MWD_ENTRY(K7V, float, 1, 16, 1), MWD_ENTRY(K7V, float, 1, 4, 4),
    // ten rows: 156 VGPRs leave three waves per SIMD, room for a ten-wave workgroup
    MWD_ENTRY(K7V, float, 1, 10, 1),
};

void mwd_table_7v_f32(const MwdEntry** tab, int* n)
{
    *tab = kEntries;
    *n = (int)(sizeof(kEntries) / sizeof(kEntries[0]));
}

}  // namespace mwd
