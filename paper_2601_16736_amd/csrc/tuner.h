// Schedule tuner table (internal).
#pragma once

#include <stdint.h>

namespace gs {

// Fastest (schedule, unit) recorded for the bucket of (n, visible fraction,
// moment dtype); false if the bucket has no entry.
bool tuner_lookup(int64_t n, float visible_fraction, int dtype, int* sched, int* unit);
void tuner_record(int64_t n, float visible_fraction, int dtype, int sched, int unit);

}  // namespace gs
