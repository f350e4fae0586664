// HBM stream probe (instrumentation, not part of the method): plain streaming
// kernels that read, write, copy or mix whole buffers, so that the rates the
// stepping kernels reach can be set beside what simple streams reach on the
// same device.  Each thread walks the buffer with a grid stride, 16 bytes per
// access; blocks of 256 threads, a chosen number per compute unit.
#include <exception>
#include <new>

#include "common.hpp"

namespace aafwi {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_probe_read(const f4* __restrict__ a, long long n, float* __restrict__ sink) {
    f4 s = {0.f, 0.f, 0.f, 0.f};
    const long long step = (long long)gridDim.x * blockDim.x;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += step) s += a[i];
    // never true for finite data of the probe; keeps the loads
    if (s.x + s.y + s.z + s.w == -1.0e38f) sink[0] = s.x;
}

__global__ __launch_bounds__(256) void k_probe_write(f4* __restrict__ b, long long n) {
    const long long step = (long long)gridDim.x * blockDim.x;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += step) b[i] = f4{1.f, 2.f, 3.f, 4.f};
}

__global__ __launch_bounds__(256) void k_probe_copy(const f4* __restrict__ a, f4* __restrict__ b, long long n) {
    const long long step = (long long)gridDim.x * blockDim.x;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += step) b[i] = a[i];
}

__global__ __launch_bounds__(256) void k_probe_mix(const f4* __restrict__ a, const f4* __restrict__ c,
                                                   f4* __restrict__ b, long long n) {
    const long long step = (long long)gridDim.x * blockDim.x;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += step) b[i] = a[i] + 2.0f * c[i];
}

}  // namespace
}  // namespace aafwi

extern "C" int aafwi_stream_probe(aafwi_stream stream, int32_t kind, int64_t bytes, int32_t blocks_per_cu,
                                  const void* a, void* b, const void* c) {
    try {
        AAFWI_REQUIRE(kind >= 0 && kind <= 3, "stream_probe: kind must be 0..3");
        AAFWI_REQUIRE(bytes > 0 && bytes % 16 == 0, "stream_probe: bytes must be a positive multiple of 16");
        AAFWI_REQUIRE(blocks_per_cu >= 1 && blocks_per_cu <= 64, "stream_probe: blocks_per_cu must be 1..64");
        AAFWI_REQUIRE(kind == 1 || a, "stream_probe: a is required");
        AAFWI_REQUIRE(b, "stream_probe: b is required");
        AAFWI_REQUIRE(kind != 3 || c, "stream_probe: c is required");
        const long long n = bytes / 16;
        const dim3 grid(256 * blocks_per_cu), block(256);
        const hipStream_t st = (hipStream_t)stream;
        using namespace aafwi;
        switch (kind) {
            case 0: hipLaunchKernelGGL(k_probe_read, grid, block, 0, st, (const f4*)a, n, (float*)b); break;
            case 1: hipLaunchKernelGGL(k_probe_write, grid, block, 0, st, (f4*)b, n); break;
            case 2: hipLaunchKernelGGL(k_probe_copy, grid, block, 0, st, (const f4*)a, (f4*)b, n); break;
            default: hipLaunchKernelGGL(k_probe_mix, grid, block, 0, st, (const f4*)a, (const f4*)c, (f4*)b, n); break;
        }
        AAFWI_HIP(hipGetLastError());
        return AAFWI_OK;
    } catch (const aafwi::Error& e) {
        aafwi::set_last_error(e.msg);
        return e.code;
    } catch (...) {
        aafwi::set_last_error("unknown error");
        return AAFWI_E_INVALID;
    }
}
