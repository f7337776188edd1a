// Calibration kernel for HBM traffic counters: a plain streaming copy of a
// known number of bytes, so that the FETCH_SIZE / WRITE_SIZE counters read
// for it give the scale between counter units and bytes moved.
#include <hip/hip_runtime.h>

#include "pic.h"

namespace {

__global__ __launch_bounds__(256) void k_copy_calibration(const float4* __restrict__ src,
                                                          float4* __restrict__ dst, long long n)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = src[i];
}

}  // namespace

extern "C" int pic_copy_calibration(int64_t bytes, int32_t reps, double* ms_per_copy)
{
    if (bytes <= 0 || bytes % 16 != 0 || reps <= 0 || !ms_per_copy) return PIC_E_INVAL;
    void* a = nullptr;
    void* b = nullptr;
    if (hipMalloc(&a, (size_t)bytes) != hipSuccess) return PIC_E_NOMEM;
    if (hipMalloc(&b, (size_t)bytes) != hipSuccess) {
        (void)hipFree(a);
        return PIC_E_NOMEM;
    }
    int rc = PIC_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const long long n = bytes / 16;
    const int grid = 256 * 8 * 4;   // 4 workgroups of 256 per SIMD-group, grid-stride
    if (hipMemsetAsync(a, 0, (size_t)bytes, 0) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        rc = PIC_E_DEVICE;
    } else {
        hipLaunchKernelGGL(k_copy_calibration, dim3(grid), dim3(256), 0, 0, (const float4*)a,
                           (float4*)b, n);
        (void)hipEventRecord(e0, 0);
        for (int r = 0; r < reps; ++r)
            hipLaunchKernelGGL(k_copy_calibration, dim3(grid), dim3(256), 0, 0, (const float4*)a,
                               (float4*)b, n);
        (void)hipEventRecord(e1, 0);
        float ms = 0.0f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            rc = PIC_E_DEVICE;
        *ms_per_copy = (double)ms / reps;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(a);
    (void)hipFree(b);
    return rc;
}
