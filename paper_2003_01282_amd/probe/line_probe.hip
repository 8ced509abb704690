// Diagnostic (not part of the SLQ path): read throughput of random 128-byte
// lines against the working-set size, the ceiling of a gather-bound SpMM
// whose rows miss L2.  Eight lanes read one line (16 bytes each), eight
// independent lines in flight per lane; line ids come from a 32-bit integer
// hash, so every line of the set is equally likely.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace {

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

__global__ void __launch_bounds__(256) line_reads(const float4* __restrict__ buf, uint32_t nlines, int iters,
                                                  uint32_t salt, float* __restrict__ sink) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t grp = tid >> 3, sub = tid & 7;
    float acc = 0.0f;
    for (int it = 0; it < iters; it += 8) {
        float4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t line = mix32(grp * 977u + (uint32_t)(it + u) * 0x9E3779B9u + salt) % nlines;
            v[u] = buf[(size_t)line * 8 + sub];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u].x + v[u].y + v[u].z + v[u].w;
    }
    sink[tid] = acc;
}

}  // namespace

extern "C" {

// For each working-set size sizes[i] (bytes, <= the largest, multiple of 128)
// reads random lines of one buffer and writes the rate in TB/s (line bytes
// per second) to tbps[i].  Allocates its buffer; returns 0 or a hipError_t.
int slaq_line_probe(const size_t* sizes, int nsizes, double* tbps) {
    size_t maxb = 0;
    for (int i = 0; i < nsizes; ++i) maxb = sizes[i] > maxb ? sizes[i] : maxb;
    if (maxb < 128 || maxb / 128 > 0xFFFFFFFFull) return (int)hipErrorInvalidValue;
    const int blocks = 8192, threads = 256, iters = 64, reps = 5;
    float4* buf = nullptr;
    float* sink = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipMalloc(&buf, maxb);
    if (e == hipSuccess) e = hipMalloc(&sink, sizeof(float) * blocks * threads);
    if (e == hipSuccess) e = hipMemset(buf, 0, maxb);
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    for (int i = 0; i < nsizes && e == hipSuccess; ++i) {
        const uint32_t nlines = (uint32_t)(sizes[i] / 128);
        if (nlines == 0) {
            e = hipErrorInvalidValue;
            break;
        }
        hipLaunchKernelGGL(line_reads, dim3(blocks), dim3(threads), 0, 0, buf, nlines, iters, 1234u, sink);
        e = hipEventRecord(a, 0);
        for (int r = 0; r < reps && e == hipSuccess; ++r) {
            hipLaunchKernelGGL(line_reads, dim3(blocks), dim3(threads), 0, 0, buf, nlines, iters, 777u * (r + 1),
                               sink);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(b, 0);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        const double bytes = (double)blocks * threads / 8 * iters * 128.0 * reps;
        tbps[i] = e == hipSuccess ? bytes / (ms * 1e-3) / 1e12 : 0.0;
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (sink) (void)hipFree(sink);
    if (buf) (void)hipFree(buf);
    return (int)e;
}

}  // extern "C"
