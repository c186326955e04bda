// Relocation select + state reset (placeholder until the select kernels land).
#include "internal.h"

namespace gs {
gs_status set_error(gs_status s, const char* msg);
}

extern "C" {

size_t gs_relocate_workspace_size(int64_t) { return 0; }

gs_status gs_relocate_reset(const float*, int64_t, int64_t, const gs_group*, int32_t, int32_t, int32_t*, int32_t,
                            int32_t*, void*, size_t, hipStream_t)
{
    return gs::set_error(GS_EUNSUPPORTED, "gs_relocate_reset: not built yet");
}

}
