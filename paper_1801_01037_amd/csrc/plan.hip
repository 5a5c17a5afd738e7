// Circuit planning (placeholder until the tile pass lands).
#include "plan.h"

namespace svk {

sv_status plan_run(sv_state, const sv_gate *, size_t, uint32_t, std::string *err)
{
    *err = "fused execution is not built yet";
    return SV_EUNSUPPORTED;
}

void plan_release(sv_state) {}

}  // namespace svk
