// Circuit planning: fusion of gate runs into passes, and their execution.
#pragma once

#include <string>

#include "sv_internal.h"

namespace svk {

// Plans and queues a validated gate list with SV_FUSE / SV_FUSE_DENSE /
// SV_GRAPH. On failure returns a status and sets *err.
sv_status plan_run(sv_state s, const sv_gate *gates, size_t n_gates, uint32_t flags,
                   std::string *err);

// Frees planning buffers and cached graphs owned by the handle.
void plan_release(sv_state s);

}  // namespace svk
