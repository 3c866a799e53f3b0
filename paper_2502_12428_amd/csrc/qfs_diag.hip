// Diagnostics: the int8 matrix-core rate this device sustains on a pure
// v_mfma_i32_16x16x64_i8 loop (register operands, eight independent
// accumulator chains per wave, no memory traffic), the ceiling the deep
// kernels' executed-MFMA figure is compared with next to the nominal peak.
#include <hip/hip_runtime.h>

#include "qfs_device.h"
#include "qfs_internal.h"

namespace qfs {

constexpr int PEAK_NT = 256, PEAK_CHAINS = 8;

__global__ __launch_bounds__(PEAK_NT) void k_mfma_peak(int iters, int *sink)
{
    const int lane = threadIdx.x & 63;
    const v4i a = v4i{lane, lane + 1, lane + 2, lane + 3}, b = v4i{3 * lane, lane ^ 5, lane + 7, 11};
    v4i acc[PEAK_CHAINS];
#pragma unroll
    for (int j = 0; j < PEAK_CHAINS; ++j) acc[j] = v4i{j, 0, 0, 0};
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < PEAK_CHAINS; ++j) acc[j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, acc[j], 0, 0, 0);
    }
    int s = 0;
#pragma unroll
    for (int j = 0; j < PEAK_CHAINS; ++j) s += acc[j].x + acc[j].y + acc[j].z + acc[j].w;
    if (s == 0x7fffffff) sink[0] = s;  // keeps the loop live; never taken for these operands
}

hipError_t mfma_peak(int iters, int nwg, int *sink, float *ms, hipStream_t s)
{
    hipEvent_t e0, e1;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return e;
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        hipEventDestroy(e0);
        return e;
    }
    hipLaunchKernelGGL(k_mfma_peak, dim3(nwg), dim3(PEAK_NT), 0, s, 1, sink);  // warm-up
    hipEventRecord(e0, s);
    hipLaunchKernelGGL(k_mfma_peak, dim3(nwg), dim3(PEAK_NT), 0, s, iters, sink);
    hipEventRecord(e1, s);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return e;
}

int64_t mfma_peak_ops(int iters, int nwg)
{
    // 16 x 16 x 64 multiply-adds (two operations each) per instruction
    return (int64_t)nwg * (PEAK_NT / 64) * iters * PEAK_CHAINS * 16 * 16 * 64 * 2;
}

}  // namespace qfs
