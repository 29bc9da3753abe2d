// Measurement only: streaming kernels that calibrate the rates the memory
// system reaches on this GPU, beside the nominal HBM peak.
//
// ce_stream_copy: the buffer is split into `streams` equal parts that one
// kernel reads and writes side by side (four parts: the two fields'
// deviation and derivative arrays that a step pass streams), with 128-bit
// loads and nontemporal stores, one load per part in flight per thread.
//
// ce_stream_probe: read+write, read-only and write-only streams with
// `unroll` independent 128-bit loads per part issued by each thread before
// its first store (so up to parts x unroll loads are in flight per thread),
// and a choice of nontemporal loads and stores.  The best of these over a
// sweep of grids is the ceiling a streaming kernel can reach.
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

template <bool NT>
__device__ __forceinline__ f32x4 probe_load(const f32x4 *p)
{
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}
template <bool NT>
__device__ __forceinline__ void probe_store(f32x4 v, f32x4 *p)
{
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// One iteration of a block covers U consecutive 256-vector segments of every
// part; vector j of part s is element s * per + j.  Indices past `per` are
// skipped, so any per works.
template <int KIND, int P, int U, bool NTL, bool NTS>
__global__ __launch_bounds__(256) void stream_probe_kernel(const f32x4 *__restrict__ src, f32x4 *__restrict__ dst,
                                                           long long per)
{
    const long long span = (long long)U * 256;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (long long base = (long long)blockIdx.x * span; base < per; base += (long long)gridDim.x * span) {
        if constexpr (KIND == CE_PROBE_WRITE) {
            const f32x4 v = {1.f, 2.f, 3.f, 4.f};
#pragma unroll
            for (int s = 0; s < P; s++)
#pragma unroll
                for (int u = 0; u < U; u++) {
                    const long long j = base + u * 256 + threadIdx.x;
                    if (j < per) probe_store<NTS>(v, &dst[(long long)s * per + j]);
                }
        } else {
            f32x4 v[P][U];
#pragma unroll
            for (int s = 0; s < P; s++)
#pragma unroll
                for (int u = 0; u < U; u++) {
                    const long long j = base + u * 256 + threadIdx.x;
                    v[s][u] = j < per ? probe_load<NTL>(&src[(long long)s * per + j]) : f32x4{0.f, 0.f, 0.f, 0.f};
                }
#pragma unroll
            for (int s = 0; s < P; s++)
#pragma unroll
                for (int u = 0; u < U; u++) {
                    const long long j = base + u * 256 + threadIdx.x;
                    if constexpr (KIND == CE_PROBE_COPY) {
                        if (j < per) probe_store<NTS>(v[s][u], &dst[(long long)s * per + j]);
                    } else {
                        acc += v[s][u];
                    }
                }
        }
    }
    if constexpr (KIND == CE_PROBE_READ) dst[(long long)blockIdx.x * 256 + threadIdx.x] = acc;
}

template <int KIND, int P, int U>
hipError_t probe_nt(const f32x4 *src, f32x4 *dst, long long per, int nt, int grid, hipStream_t st)
{
    switch (nt) {
    case 0: hipLaunchKernelGGL((stream_probe_kernel<KIND, P, U, false, false>), dim3(grid), dim3(256), 0, st, src, dst, per); break;
    case 1: hipLaunchKernelGGL((stream_probe_kernel<KIND, P, U, true, false>), dim3(grid), dim3(256), 0, st, src, dst, per); break;
    case 2: hipLaunchKernelGGL((stream_probe_kernel<KIND, P, U, false, true>), dim3(grid), dim3(256), 0, st, src, dst, per); break;
    case 3: hipLaunchKernelGGL((stream_probe_kernel<KIND, P, U, true, true>), dim3(grid), dim3(256), 0, st, src, dst, per); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int KIND, int P>
hipError_t probe_unroll(const f32x4 *src, f32x4 *dst, long long per, int unroll, int nt, int grid, hipStream_t st)
{
    switch (unroll) {
    case 1: return probe_nt<KIND, P, 1>(src, dst, per, nt, grid, st);
    case 2: return probe_nt<KIND, P, 2>(src, dst, per, nt, grid, st);
    case 4: return probe_nt<KIND, P, 4>(src, dst, per, nt, grid, st);
    case 8: return probe_nt<KIND, P, 8>(src, dst, per, nt, grid, st);
    default: return hipErrorInvalidValue;
    }
}

template <int KIND>
hipError_t probe_parts(const f32x4 *src, f32x4 *dst, long long per, int parts, int unroll, int nt, int grid,
                       hipStream_t st)
{
    switch (parts) {
    case 1: return probe_unroll<KIND, 1>(src, dst, per, unroll, nt, grid, st);
    case 4: return probe_unroll<KIND, 4>(src, dst, per, unroll, nt, grid, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_probe(int kind, const f32x4 *src, f32x4 *dst, long long per, int parts, int unroll, int nt,
                        int grid, hipStream_t st)
{
    switch (kind) {
    case CE_PROBE_COPY: return probe_parts<CE_PROBE_COPY>(src, dst, per, parts, unroll, nt, grid, st);
    case CE_PROBE_READ: return probe_parts<CE_PROBE_READ>(src, dst, per, parts, unroll, nt, grid, st);
    case CE_PROBE_WRITE: return probe_parts<CE_PROBE_WRITE>(src, dst, per, parts, unroll, nt, grid, st);
    default: return hipErrorInvalidValue;
    }
}

// Time `reps` launches of `launch` on `st` after one warm-up launch.
template <typename F>
ce_status time_launches(F &&launch, int reps, hipStream_t st, float *ms)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    CE_HIP(hipEventCreate(&e0));
    hipError_t err = hipEventCreate(&e1);
    if (err == hipSuccess) err = launch();  // warm-up
    if (err == hipSuccess) err = hipEventRecord(e0, st);
    for (int r = 0; r < reps && err == hipSuccess; r++) err = launch();
    if (err == hipSuccess) err = hipEventRecord(e1, st);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float t = 0.0f;
    if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (err != hipSuccess) return fail(CE_EDEVICE, "measurement stream failed: %s", hipGetErrorString(err));
    *ms = t / (float)reps;
    return CE_OK;
}

ce_status default_grid(int32_t *grid)
{
    if (*grid != 0) return CE_OK;
    int cus = 0;
    const ce_status st = device_cus(&cus);
    if (st != CE_OK) return st;
    *grid = 16 * cus;
    return CE_OK;
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
    const ce_status gs = default_grid(&grid);
    if (gs != CE_OK) return gs;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const long long per = (long long)(bytes / 16 / (size_t)streams);
    const f32x4 *s = static_cast<const f32x4 *>(src);
    f32x4 *d = static_cast<f32x4 *>(dst);
    return time_launches([&] { return launch_copy(s, d, per, streams, grid, st); }, reps, st, ms);
}

extern "C" ce_status ce_stream_probe(int32_t kind, const void *src, void *dst, size_t bytes, int32_t parts,
                                     int32_t unroll, int32_t nt, int32_t grid, int32_t reps, void *stream,
                                     float *ms)
{
    if (!ms) return fail(CE_EINVAL, "NULL argument");
    if (kind != CE_PROBE_COPY && kind != CE_PROBE_READ && kind != CE_PROBE_WRITE)
        return fail(CE_EINVAL, "kind must be CE_PROBE_COPY, CE_PROBE_READ or CE_PROBE_WRITE");
    if ((kind != CE_PROBE_WRITE && !src) || !dst) return fail(CE_EINVAL, "NULL buffer");
    if (parts != 1 && parts != 4) return fail(CE_EINVAL, "parts must be 1 or 4");
    if (unroll != 1 && unroll != 2 && unroll != 4 && unroll != 8) return fail(CE_EINVAL, "unroll must be 1, 2, 4 or 8");
    if (nt < 0 || nt > 3) return fail(CE_EINVAL, "nt must be 0..3");
    if (bytes == 0 || bytes % (16u * (size_t)parts)) return fail(CE_EINVAL, "bytes must be a multiple of 16 * parts");
    if ((uintptr_t)src % 16 || (uintptr_t)dst % 16) return fail(CE_EINVAL, "buffers must be 16-byte aligned");
    if (grid < 0 || grid > (1 << 20) || reps < 1) return fail(CE_EINVAL, "grid must be 0..2^20 and reps >= 1");
    const ce_status gs = default_grid(&grid);
    if (gs != CE_OK) return gs;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const long long per = (long long)(bytes / 16 / (size_t)parts);
    // the read-only kernel writes one vector per thread into dst
    if (kind == CE_PROBE_READ && (unsigned long long)grid * 256ull * 16ull > bytes)
        return fail(CE_EINVAL, "read probe: dst must hold grid * 256 vectors (at most `bytes`)");
    const f32x4 *s = static_cast<const f32x4 *>(src);
    f32x4 *d = static_cast<f32x4 *>(dst);
    return time_launches([&] { return launch_probe(kind, s, d, per, parts, unroll, nt, grid, st); }, reps, st, ms);
}
