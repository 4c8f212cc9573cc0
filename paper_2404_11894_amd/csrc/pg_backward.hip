// pg_backward.hip -- reverse mode of the render (albedo grid and HG g).
#include "pg_api_common.h"

using namespace pg;

extern "C" {

pg_status pg_backward_workspace_size(const pg_paths* paths, const pg_params* params, size_t* bytes) {
    (void)paths; (void)params; (void)bytes;
    return fail(PG_ERR_UNSUPPORTED, "pg_backward: not built yet");
}

pg_status pg_backward(const pg_paths* paths, const pg_params* params, const float* grad_image, float* grad_grid,
                      float* grad_albedo, float* grad_g, void* ws, size_t ws_bytes, void* stream) {
    (void)paths; (void)params; (void)grad_image; (void)grad_grid; (void)grad_albedo; (void)grad_g;
    (void)ws; (void)ws_bytes; (void)stream;
    return fail(PG_ERR_UNSUPPORTED, "pg_backward: not built yet");
}

}  // extern "C"
