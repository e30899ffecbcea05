// Host-memory stand-ins for the HIP runtime calls of the geometry
// preprocessor and batch planner, and empty launchers, so that those run
// unchanged on a CPU for the tests (device memory = host memory).
#include <cstdlib>
#include <cstring>

#include "gt_internal.h"

extern "C" {
hipError_t hipMalloc(void **p, size_t n) {
    *p = std::calloc(1, n ? n : 1);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void *p) {
    std::free(p);
    return hipSuccess;
}
hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) {
    std::memcpy(d, s, n);
    return hipSuccess;
}
hipError_t hipGetDevice(int *d) {
    *d = 0;
    return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
const char *hipGetErrorString(hipError_t) { return "host build"; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t *) { return hipErrorNotSupported; }
hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float *, hipEvent_t, hipEvent_t) { return hipSuccess; }
}

namespace gt {
int launch_track(const gt_geometry *, const gt_track_params *, const gt_track_out *, void *, const gt_mesh *) {
    return set_error("host build: no kernels"), GT_EHIP;
}
int launch_batch(gt_batch *, void *) { return set_error("host build: no kernels"), GT_EHIP; }
int launch_event(const gt_geometry *, const gt_track_params *, const gt_track_out *, void *, void *) {
    return set_error("host build: no kernels"), GT_EHIP;
}
int prepare_batch_streams(gt_batch *) { return GT_OK; }
void release_batch_streams(gt_batch *) {}
int launch_find_cell(const gt_geometry *, const double *, uint64_t, int64_t *, int32_t *, uint32_t, void *) {
    return GT_EHIP;
}
int launch_distance(const gt_geometry *, const double *, const double *, const int32_t *, uint64_t, double *,
                    int32_t *, int32_t *, void *) {
    return GT_EHIP;
}
int launch_fp64_check(const double *, const double *, uint64_t, double *, double *, double *, void *) {
    return GT_EHIP;
}
void set_kernel_events(void *, void *) {}
bool last_launch(gt_launch_info *) { return false; }   // no device launches here
}  // namespace gt
