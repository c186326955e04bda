// Host-side launch plumbing shared by the entry points.
//
// Launch log: with GSOPT_TRACE set (and not "0") in the environment, each
// step entry point writes one line to stderr describing the launch it makes.
// The variable is read at every call.
#pragma once

#include <cstdint>

#include "gsopt.h"

namespace gs {

bool trace_on();

// detail: what else the entry point wants logged (camera or scene count)
void trace_step(const char* entry, int64_t n, int n_groups, const char* schedule, int unit,
                const gs_step_config* cfg, const char* detail);

// A dispatch holds at most 2^32 - 1 work-items.  One wave per unit of `unit`
// rows over `rows` rows needs more than that only for the 32-row units of the
// largest scenes (rows > 2^31 - 128); the smallest unit size from `unit` up
// to `max_unit` that fits is returned (every unit size gives the same bits).
int fit_unit(int64_t rows, int unit, int max_unit);

// Largest grid (blocks of 256 threads) one dispatch can hold.
constexpr int64_t kMaxGridBlocks = 0xFFFFFFFFll / 256;

}  // namespace gs
