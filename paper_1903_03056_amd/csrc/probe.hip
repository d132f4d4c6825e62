// Attainable FP32 vector throughput of the device, for stating roofline fractions
// against a measured ceiling next to the datasheet one: a grid of waves each running
// eight independent FMA chains, timed with HIP events.  The library is built without
// packed FP32, so this is the ceiling of the unpacked FMA the kernels use.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dgfs.h"

namespace {

constexpr int kChains = 8;

__global__ __launch_bounds__(256) void fma_chains(float* out, int iters, float b, float c) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    float a[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = float(t + k) * 1e-7f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) a[k] = fmaf(a[k], b, c);
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += a[k];
    out[t] = s;
}

}  // namespace

extern "C" dgfs_status dgfs_probe_valu(void* scratch, size_t scratch_bytes, int32_t blocks, int32_t iters,
                                       void* stream, double* tflops) {
    if (!scratch || !tflops || blocks < 1 || iters < 1) return DGFS_EINVAL;
    if (scratch_bytes < size_t(blocks) * 256 * sizeof(float)) return DGFS_ENOMEM;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return DGFS_EDEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return DGFS_EDEVICE;
    }
    float* out = static_cast<float*>(scratch);
    fma_chains<<<dim3(unsigned(blocks)), dim3(256), 0, st>>>(out, iters, 0.999999f, 1e-6f);  // warm-up
    hipEventRecord(e0, st);
    fma_chains<<<dim3(unsigned(blocks)), dim3(256), 0, st>>>(out, iters, 0.999999f, 1e-6f);
    hipEventRecord(e1, st);
    dgfs_status rc = DGFS_OK;
    float ms = 0.0f;
    if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess || ms <= 0.0f) {
        rc = DGFS_EDEVICE;
    } else {
        const double flops = 2.0 * kChains * double(iters) * double(blocks) * 256.0;
        *tflops = flops / (double(ms) * 1e-3) / 1e12;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return rc;
}
