// pvfind_compact.hip -- output compaction for transfers: the written vertex
// records of a batch (n_vertices[e] of the max_vertices slots of each event)
// gathered into one dense array, so that only they cross PCIe.
#include <hip/hip_runtime.h>

#include "pvfind_internal.h"

namespace pvk {

constexpr int kScanThreads = 1024;

// first[e] = sum of n_vertices over the events before e, first[n_events] the
// total: one workgroup, each thread scans a contiguous run of events.
// Negative counts (an event skipped before it wrote one) count as 0.
__global__ __launch_bounds__(kScanThreads) void vertex_prefix_kernel(const int32_t *nv, const int32_t *n_events_dev,
                                                                     int n_events_host, int max_v, int32_t *first)
{
    __shared__ int part[kScanThreads];
    const int tid = threadIdx.x;
    const int n_events = n_events_dev ? *n_events_dev : n_events_host;
    const int per = (n_events + kScanThreads - 1) / kScanThreads;
    const int a = min(n_events, tid * per), b = min(n_events, a + per);
    int s = 0;
    for (int e = a; e < b; ++e)
        s += min(max(nv[e], 0), max_v);
    part[tid] = s;
    __syncthreads();
    // inclusive scan of the per-thread sums (Hillis-Steele over LDS)
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const int v = (tid >= off) ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int run = part[tid] - s;
    for (int e = a; e < b; ++e) {
        first[e] = run;
        run += min(max(nv[e], 0), max_v);
    }
    if (tid == kScanThreads - 1)
        first[n_events] = part[tid];
}

// four threads per event, each moving one 16-byte quarter of each record
__global__ __launch_bounds__(256) void vertex_gather_kernel(const pv_vertex *slots, const int32_t *nv,
                                                            const int32_t *n_events_dev, int n_events_host, int max_v,
                                                            const int32_t *first, pv_vertex *dense)
{
    const int n_events = n_events_dev ? *n_events_dev : n_events_host;
    const int t = blockIdx.x * 256 + threadIdx.x;
    const int e = t >> 2, q = t & 3;
    if (e >= n_events)
        return;
    const int n = min(max(nv[e], 0), max_v);
    const uint4 *src = reinterpret_cast<const uint4 *>(slots + (size_t)e * max_v);
    uint4 *dst = reinterpret_cast<uint4 *>(dense + first[e]);
    for (int v = 0; v < n; ++v)
        dst[4 * v + q] = src[4 * v + q];
}

// The two launches; with n_events_dev the count is read from device memory
// and n_events is its upper bound (the grid size).
int launch_compact(const pv_vertex *slots, const int32_t *nv, const int32_t *n_events_dev, int n_events, int max_v,
                   pv_vertex *dense, int32_t *first, void *stream)
{
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(vertex_prefix_kernel, dim3(1), dim3(kScanThreads), 0, st, nv, n_events_dev, n_events, max_v,
                       first);
    hipError_t err = hipGetLastError();
    if (err == hipSuccess && n_events > 0) {
        const int grid = (4 * n_events + 255) / 256;
        hipLaunchKernelGGL(vertex_gather_kernel, dim3(grid), dim3(256), 0, st, slots, nv, n_events_dev, n_events, max_v,
                           first, dense);
        err = hipGetLastError();
    }
    return (int)err;
}

}  // namespace pvk

extern "C" int pv_compact_vertices(const pv_vertex *slots, const int32_t *n_vertices, int32_t n_events,
                                   int32_t max_vertices, pv_vertex *dense, int32_t *first, void *stream)
{
    using namespace pvk;
    if (!slots || !n_vertices || !dense || !first)
        return set_error(PV_EINVAL, "pv_compact_vertices: null pointer");
    if (n_events < 0 || max_vertices < 1 || max_vertices > kMaxVertices)
        return set_error(PV_EINVAL, "pv_compact_vertices: n_events %d / max_vertices %d out of range", n_events,
                         max_vertices);
    const hipError_t err = (hipError_t)launch_compact(slots, n_vertices, nullptr, n_events, max_vertices, dense, first,
                                                      stream);
    if (err != hipSuccess)
        return set_error(PV_EHIP, "pv_compact_vertices: %s", hipGetErrorString(err));
    return PV_OK;
}
