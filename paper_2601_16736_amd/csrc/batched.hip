// Many scenes in one persistent launch (placeholder until the plan kernel lands).
#include "internal.h"

namespace gs {
gs_status set_error(gs_status s, const char* msg);
}

extern "C" {

gs_status gs_batch_create(const gs_scene*, int32_t, gs_batch** out)
{
    if (out) *out = nullptr;
    return gs::set_error(GS_EUNSUPPORTED, "gs_batch_create: not built yet");
}

gs_status adamw_gs_step_batched(gs_batch*, const gs_step_config*, hipStream_t)
{
    return gs::set_error(GS_EUNSUPPORTED, "adamw_gs_step_batched: not built yet");
}

int32_t gs_batch_scene_schedule(const gs_batch*, int32_t) { return -1; }

gs_status gs_batch_destroy(gs_batch*) { return GS_OK; }

}
