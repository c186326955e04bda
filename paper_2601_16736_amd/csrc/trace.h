// Launch log of the step entry points: with GSOPT_TRACE set (and not "0")
// in the environment, each entry point writes one line to stderr describing
// the launch it makes.  The variable is read at every call.
#pragma once

#include <cstdint>

#include "gsopt.h"

namespace gs {

bool trace_on();

// detail: what else the entry point wants logged (camera or scene count)
void trace_step(const char* entry, int64_t n, int n_groups, const char* schedule, int unit,
                const gs_step_config* cfg, const char* detail);

}  // namespace gs
