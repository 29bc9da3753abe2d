// Measurement only: a streaming copy that calibrates the read+write rate the
// memory system reaches on this GPU, beside the nominal HBM peak.  The buffer
// is split into `streams` equal parts that one kernel reads and writes side
// by side (four parts: the two fields' deviation and derivative arrays that a
// step pass streams), with 128-bit loads and nontemporal stores.
#include <hip/hip_runtime.h>

#include "ce_sim.hpp"

using namespace ce;
using namespace ce::host;

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int S>
__global__ __launch_bounds__(256) void stream_copy_kernel(const f32x4 *__restrict__ src, f32x4 *__restrict__ dst,
                                                          long long per)
{
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < per; i += (long long)gridDim.x * 256) {
        f32x4 v[S];
#pragma unroll
        for (int s = 0; s < S; s++) v[s] = src[(long long)s * per + i];
#pragma unroll
        for (int s = 0; s < S; s++) __builtin_nontemporal_store(v[s], &dst[(long long)s * per + i]);
    }
}

hipError_t launch_copy(const f32x4 *src, f32x4 *dst, long long per, int streams, int grid, hipStream_t st)
{
    switch (streams) {
    case 1: hipLaunchKernelGGL((stream_copy_kernel<1>), dim3(grid), dim3(256), 0, st, src, dst, per); break;
    case 2: hipLaunchKernelGGL((stream_copy_kernel<2>), dim3(grid), dim3(256), 0, st, src, dst, per); break;
    case 4: hipLaunchKernelGGL((stream_copy_kernel<4>), dim3(grid), dim3(256), 0, st, src, dst, per); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

extern "C" ce_status ce_stream_copy(const void *src, void *dst, size_t bytes, int32_t streams, int32_t grid,
                                    int32_t reps, void *stream, float *ms)
{
    if (!src || !dst || !ms) return fail(CE_EINVAL, "NULL argument");
    if (streams != 1 && streams != 2 && streams != 4) return fail(CE_EINVAL, "streams must be 1, 2 or 4");
    if (bytes == 0 || bytes % (16u * (size_t)streams)) return fail(CE_EINVAL, "bytes must be a multiple of 16 * streams");
    if ((uintptr_t)src % 16 || (uintptr_t)dst % 16) return fail(CE_EINVAL, "buffers must be 16-byte aligned");
    if (grid < 0 || reps < 1) return fail(CE_EINVAL, "grid must be >= 0 and reps >= 1");
    if (grid == 0) {
        int cus = 0;
        const ce_status st = device_cus(&cus);
        if (st != CE_OK) return st;
        grid = 16 * cus;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const long long per = (long long)(bytes / 16 / (size_t)streams);
    const f32x4 *s = static_cast<const f32x4 *>(src);
    f32x4 *d = static_cast<f32x4 *>(dst);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    CE_HIP(hipEventCreate(&e0));
    hipError_t err = hipEventCreate(&e1);
    if (err == hipSuccess) err = launch_copy(s, d, per, streams, grid, st);  // warm-up
    if (err == hipSuccess) err = hipEventRecord(e0, st);
    for (int r = 0; r < reps && err == hipSuccess; r++) err = launch_copy(s, d, per, streams, grid, st);
    if (err == hipSuccess) err = hipEventRecord(e1, st);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float t = 0.0f;
    if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (err != hipSuccess) return fail(CE_EDEVICE, "stream copy failed: %s", hipGetErrorString(err));
    *ms = t / (float)reps;
    return CE_OK;
}
