// The memory coalescing experiment (Ch.2, "Memory coalescing experiment"),
// as a measurement of the attainable bandwidth of the GPU the library runs
// on: every element of an array is read and written once (x += 8) by a
// grid-stride loop, with the elements that the lanes of one wavefront touch
// spread over C arrays (C = 1: one contiguous run per wavefront, fully
// coalesced; C = 64: every lane in a different 1/64 of the array).  The
// thesis's form has 32-lane warps; here the SIMD width is 64.
#include <hip/hip_runtime.h>

#include "smmo_host.hpp"

namespace {

__global__ __launch_bounds__(256) void k_coalescing(float *data, uint64_t n, uint32_t C)
{
    const uint32_t seg = 64u / C;               // lanes per contiguous segment
    const uint64_t part = n / C;                // elements per array
    for (uint64_t tid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; tid < n;
         tid += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t index = ((tid % 64) / seg) * part + (tid / 64) * seg + tid % seg;
        data[index] += 8.0f;
    }
}

} // namespace

smmo_status smmo_coalescing_probe(float *data, uint64_t n, uint32_t C, uint32_t grid, smmo_stream stream)
{
    if (!data) return smmo::fail(SMMO_EINVAL, "coalescing probe: data is NULL");
    if (C == 0 || C > 64 || (C & (C - 1))) return smmo::fail(SMMO_EINVAL, "coalescing probe: C must be 1, 2, 4 .. 64");
    if (n == 0 || n % (64ull * C)) return smmo::fail(SMMO_EINVAL, "coalescing probe: n must be a multiple of 64 * C");
    if (grid == 0) grid = 2048;
    hipLaunchKernelGGL(k_coalescing, dim3(grid), dim3(256), 0, static_cast<hipStream_t>(stream), data, n, C);
    return smmo::heap_launch_check("k_coalescing");
}
