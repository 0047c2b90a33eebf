// Host lookup of the compiled MWD instantiations (one table per kind and dtype,
// built by the mwd_inst_*.hip files).
#include "mwd_rows.hpp"

namespace mwd {

#define MWD_TABLE_DECL(NAME) void NAME(const MwdEntry** tab, int* n);
MWD_TABLE_DECL(mwd_table_7c_f64)
MWD_TABLE_DECL(mwd_table_7c_f32)
MWD_TABLE_DECL(mwd_table_7v_f64)
MWD_TABLE_DECL(mwd_table_7v_f32)
MWD_TABLE_DECL(mwd_table_25c_f64)
MWD_TABLE_DECL(mwd_table_25c_f32)
MWD_TABLE_DECL(mwd_table_25v_f64)
MWD_TABLE_DECL(mwd_table_25v_f32)

static const MwdEntry* find_entry(int kind, int dtype, const MwdShape& s)
{
    using TableFn = void (*)(const MwdEntry**, int*);
    static const TableFn fns[4][2] = {
        {mwd_table_7c_f64, mwd_table_7c_f32},
        {mwd_table_7v_f64, mwd_table_7v_f32},
        {mwd_table_25c_f64, mwd_table_25c_f32},
        {mwd_table_25v_f64, mwd_table_25v_f32},
    };
    if (kind < 0 || kind > 3 || dtype < 0 || dtype > 1) return nullptr;
    const MwdEntry* tab = nullptr;
    int n = 0;
    fns[kind][dtype](&tab, &n);
    for (int i = 0; i < n; ++i)
        if (tab[i].dw == s.dw && tab[i].wpr == s.wpr) return &tab[i];
    return nullptr;
}

bool mwd_supported(int kind, int dtype, const MwdShape& s) { return find_entry(kind, dtype, s) != nullptr; }

int mwd_shapes(int kind, int dtype, MwdShape* out, int cap)
{
    if (kind < 0 || kind > 3 || dtype < 0 || dtype > 1) return 0;
    static const int dws[] = {4, 8, 10, 16};
    static const int wprs[] = {1, 2, 4};
    int n = 0;
    for (int dw : dws)
        for (int wpr : wprs) {
            MwdShape s{dw, wpr};
            if (find_entry(kind, dtype, s) && n < cap) out[n++] = s;
        }
    return n;
}

hipError_t mwd_kernel_scratch(int kind, int dtype, const MwdShape& s, size_t* bytes_per_lane)
{
    const MwdEntry* e = find_entry(kind, dtype, s);
    if (!e) return hipErrorInvalidValue;
    hipFuncAttributes fa;
    hipError_t err = hipFuncGetAttributes(&fa, e->kernel);
    if (err != hipSuccess) return err;
    *bytes_per_lane = fa.localSizeBytes;
    return hipSuccess;
}

hipError_t mwd_kernel_resources(int kind, int dtype, const MwdShape& s, int out[5])
{
    const MwdEntry* e = find_entry(kind, dtype, s);
    if (!e) return hipErrorInvalidValue;
    hipFuncAttributes fa;
    hipError_t err = hipFuncGetAttributes(&fa, e->kernel);
    if (err != hipSuccess) return err;
    int per_cu = 0;
    err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, e->kernel, 64 * s.dw * s.wpr, 0);
    if (err != hipSuccess) return err;
    out[0] = fa.numRegs;
    out[1] = (int)fa.sharedSizeBytes;
    out[2] = (int)fa.localSizeBytes;
    out[3] = 64 * s.dw * s.wpr;
    out[4] = per_cu;
    return hipSuccess;
}

int mwd_levels(int kind, const MwdShape& s) { return s.dw / radius_of(kind) - 1; }

int mwd_xtile(int kind, const MwdShape& s) { return 64 * s.wpr - 2 * mwd_levels(kind, s) * radius_of(kind); }

hipError_t mwd_run(const DevGrid& g, const HostWeights& w, int T, const MwdShape& s,
                   void* const scratch[4], hipStream_t stream, Prof* prof)
{
    const MwdEntry* e = find_entry(w.kind, g.dtype, s);
    if (!e) return hipErrorInvalidValue;
    return e->fn(g, w, T, scratch, stream, prof, 0, 1 << 30);
}

hipError_t mwd_run_rows(const DevGrid& g, const HostWeights& w, int T, const MwdShape& s, void* const scratch[4],
                        hipStream_t stream, int rho_lo, int rho_hi)
{
    const MwdEntry* e = find_entry(w.kind, g.dtype, s);
    if (!e) return hipErrorInvalidValue;
    return e->fn(g, w, T, scratch, stream, nullptr, rho_lo, rho_hi);
}

}  // namespace mwd
