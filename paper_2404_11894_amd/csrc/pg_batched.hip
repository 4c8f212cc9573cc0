// pg_batched.hip -- many independent scenes per launch.
#include "pg_api_common.h"

using namespace pg;

extern "C" {

pg_status pg_render_batched_workspace_size(int32_t n_scenes, const pg_paths* paths, const pg_params* params,
                                           size_t* bytes) {
    (void)n_scenes; (void)paths; (void)params; (void)bytes;
    return fail(PG_ERR_UNSUPPORTED, "pg_render_batched: not built yet");
}

pg_status pg_render_batched(int32_t n_scenes, const pg_paths* paths, const pg_params* params,
                            float* const* images, void* ws, size_t ws_bytes, void* stream) {
    (void)n_scenes; (void)paths; (void)params; (void)images; (void)ws; (void)ws_bytes; (void)stream;
    return fail(PG_ERR_UNSUPPORTED, "pg_render_batched: not built yet");
}

}  // extern "C"
