// LDS read-bandwidth probe: the peak against which the on-chip kernels'
// state traffic is reported.  Each workgroup of 256 threads fills 32 KiB of
// LDS, then every thread reads 8 float4 per iteration at addresses that move
// with the iteration (so no load can be hoisted or merged); consecutive lanes
// read consecutive 16-byte words, so a wave's ds_read_b128 covers 1 KiB
// without bank conflicts.  The loaded values are consumed by an empty asm
// statement (no arithmetic competes with the loads) and one of them is summed,
// so that the result depends on the reads.
#include "rg_internal.h"

namespace rg {
namespace {

constexpr int WORDS = 2048;  // float4 words of LDS per workgroup (32 KiB)

__global__ void __launch_bounds__(LDS_PROBE_THREADS) k_lds_probe(float *out, int iters) {
    __shared__ float4 buf[WORDS];
    const int t = threadIdx.x;
    for (int i = t; i < WORDS; i += LDS_PROBE_THREADS)
        buf[i] = make_float4((float)i, (float)(i + 1), (float)(i + 2), (float)(i + 3));
    __syncthreads();
    float acc = 0.0f;
    int base = t;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const float4 v = buf[(base + u * LDS_PROBE_THREADS) & (WORDS - 1)];
            asm volatile("" ::"v"(v.x), "v"(v.y), "v"(v.z), "v"(v.w));
            acc += v.x;
        }
        base = (base + 8 * LDS_PROBE_THREADS + 64) & (WORDS - 1);
    }
    out[(size_t)blockIdx.x * LDS_PROBE_THREADS + t] = acc;
}

}  // namespace

hipError_t launch_lds_probe(float *out, int blocks, int iters, hipStream_t s) {
    static_assert(LDS_PROBE_BYTES_PER_THREAD_ITER == 8 * sizeof(float4), "bytes read per thread and iteration");
    hipLaunchKernelGGL(k_lds_probe, dim3(blocks), dim3(LDS_PROBE_THREADS), 0, s, out, iters);
    return hipGetLastError();
}

}  // namespace rg
