// pg_noalloc.hip -- pg_propagate_static: pg_propagate for callers that cannot
// allocate device memory.  Its workspace (input-error flag, successor ids,
// albedos and the aggregated vector y) lives in a file-scope device array of
// PG_STATIC_SCRATCH_BYTES that every call on a device shares.  Host code
// never passes the array's name to a kernel or a copy: the name is a host-side
// stand-in, and the array's device address is looked up once per device with
// hipGetSymbolAddress while that device is current.
#include <mutex>

#include "pg_api_common.h"

namespace {

static __device__ __align__(256) unsigned char scratch[PG_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device.
pg_status scratch_address(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return pg::hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return pg::fail(PG_ERR_UNSUPPORTED, "device ordinal %d outside [0, %d)", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return pg::hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return pg::fail(PG_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PG_OK;
}

}  // namespace

extern "C" pg_status pg_propagate_static(const pg_paths* paths, const pg_params* params, const int64_t* row_ptr,
                                         const int32_t* col, const float* w_ind, const float* b, float* lplus,
                                         float* traj, void* stream) {
    pg::g_error.clear();
    pg_status st;
    if ((st = pg::validate_paths(paths, false)) || (st = pg::validate_params(params)) ||
        (st = pg::no_clusters(params)))
        return st;
    const size_t need = pg::propagate_size(paths, params);
    if (need > (size_t)PG_STATIC_SCRATCH_BYTES)
        return pg::fail(PG_ERR_WORKSPACE,
                        "pg_propagate_static: N = %lld needs %zu bytes of workspace; the static scratch holds %zu "
                        "(use pg_propagate with a workspace)",
                        (long long)paths->n_vertices, need, (size_t)PG_STATIC_SCRATCH_BYTES);
    void* ws = nullptr;
    if ((st = scratch_address(&ws))) return st;
    return pg::propagate_run(paths, params, row_ptr, col, w_ind, b, lplus, traj, ws, PG_STATIC_SCRATCH_BYTES,
                             (hipStream_t)stream);
}
