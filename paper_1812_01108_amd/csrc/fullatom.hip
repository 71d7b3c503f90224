// Full-atom model: placeholder until the full-atom kernels land.
#include "a2c_internal.h"

namespace a2c {

a2c_status build_fullatom_tables(a2c_plan *p, const a2c_residue_table *table)
{
    (void)p;
    (void)table;
    set_error("full-atom model not available in this build");
    return A2C_ERR_UNSUPPORTED;
}

hipError_t launch_fa_forward_scan(const a2c_plan &, const float *, float *, hipStream_t)
{
    return hipErrorNotSupported;
}

hipError_t launch_fa_backward_scan(const a2c_plan &, const float *, const float *, const float *,
                                   float *, hipStream_t)
{
    return hipErrorNotSupported;
}

}  // namespace a2c
