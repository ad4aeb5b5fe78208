// pvfind_measure.hip -- measurement support: the LDS bandwidth the kernels of
// this library are held against (a read microbenchmark), timed with HIP
// events on the caller's stream.
#include <hip/hip_runtime.h>

#include "pvfind_internal.h"

namespace pvk {

constexpr int kLdsProbeThreads = 256;
constexpr int kLdsProbeWords = 16384;   // 64 KiB of LDS per workgroup
constexpr int kLdsProbeIters = 4096;    // 16-byte reads per thread and launch

// Every thread reads 16 bytes per step from an address that no other lane of
// its wavefront shares a bank with (consecutive lanes, consecutive 16-byte
// words; the wavefront's 1 KiB window moves by 1 KiB each step, wrapping
// inside the 64 KiB array).  The reads are folded into registers and one
// word per thread is written at the end, so none of them is dead code.
__global__ __launch_bounds__(kLdsProbeThreads) void lds_read_probe(uint32_t *sink, int iters)
{
    __shared__ uint4 buf[kLdsProbeWords / 4];
    const int tid = threadIdx.x;
    for (int i = tid; i < kLdsProbeWords / 4; i += kLdsProbeThreads)
        buf[i] = make_uint4(i, i * 3u, i * 5u, i * 7u);
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6;
    uint4 acc = make_uint4(0u, 0u, 0u, 0u);
    int idx = (wave * 64 + lane) & (kLdsProbeWords / 4 - 1);
    for (int it = 0; it < iters; ++it) {
        const uint4 v = buf[idx];
        acc.x ^= v.x;
        acc.y += v.y;
        acc.z ^= v.z;
        acc.w += v.w;
        idx = (idx + 64) & (kLdsProbeWords / 4 - 1);
    }
    sink[blockIdx.x * kLdsProbeThreads + tid] = acc.x ^ acc.y ^ acc.z ^ acc.w;
}

}  // namespace pvk

extern "C" int pv_measure_lds_peak(double *bytes_per_s, int32_t *workgroups, void *stream)
{
    using namespace pvk;
    if (!bytes_per_s)
        return set_error(PV_EINVAL, "pv_measure_lds_peak: null output");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    int dev = 0, cus = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err == hipSuccess)
        err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (err != hipSuccess)
        return set_error(PV_EHIP, "pv_measure_lds_peak: %s", hipGetErrorString(err));
    // two 64 KiB workgroups fit a CU's 160 KiB; eight waves per CU keep the
    // LDS pipes busy
    const int grid = 2 * cus;
    uint32_t *sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    err = hipMalloc(&sink, sizeof(uint32_t) * (size_t)grid * kLdsProbeThreads);
    if (err == hipSuccess)
        err = hipEventCreate(&e0);
    if (err == hipSuccess)
        err = hipEventCreate(&e1);
    float best_ms = 0.0f;
    for (int rep = 0; rep < 4 && err == hipSuccess; ++rep) {
        err = hipEventRecord(e0, st);
        if (err == hipSuccess) {
            hipLaunchKernelGGL(lds_read_probe, dim3(grid), dim3(kLdsProbeThreads), 0, st, sink, kLdsProbeIters);
            err = hipGetLastError();
        }
        if (err == hipSuccess)
            err = hipEventRecord(e1, st);
        if (err == hipSuccess)
            err = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (err == hipSuccess)
            err = hipEventElapsedTime(&ms, e0, e1);
        if (err == hipSuccess && rep > 0 && (best_ms == 0.0f || ms < best_ms))
            best_ms = ms;   // the first launch is a warm-up
    }
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    if (sink)
        (void)hipFree(sink);
    if (err != hipSuccess)
        return set_error(PV_EHIP, "pv_measure_lds_peak: %s", hipGetErrorString(err));
    const double bytes = (double)grid * kLdsProbeThreads * kLdsProbeIters * 16.0;
    *bytes_per_s = bytes / (best_ms * 1e-3);
    if (workgroups)
        *workgroups = grid;
    return PV_OK;
}
