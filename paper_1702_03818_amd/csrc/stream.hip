// Streaming copy: the HBM ceiling the stage kernels are measured against.
//
// Every lane moves 16 bytes per access (one 128-bit load and one 128-bit
// store), four independent accesses in flight per lane and iteration, over a
// grid of a few workgroups per CU that strides through the buffer; block
// indices are remapped so each XCD streams a contiguous range; plain or
// nontemporal accesses. No arithmetic: the time is the memory system's.
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace frkc2 {
namespace {

using namespace dev;

constexpr int kStreamThreads = 256;
typedef double dvec2 __attribute__((ext_vector_type(2)));   // one 128-bit access
constexpr int kUnroll = 4;

template <bool NT>
__global__ __launch_bounds__(kStreamThreads) void stream_copy(const dvec2 *__restrict__ src,
                                                              dvec2 *__restrict__ dst,
                                                              long long n)
{
    const long long nb = gridDim.x;
    const long long b = xcd_remap(blockIdx.x, gridDim.x);
    const long long chunk = (long long)kStreamThreads * kUnroll;
    for (long long base = b * chunk; base < n; base += nb * chunk) {
        dvec2 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const long long i = base + u * kStreamThreads + threadIdx.x;
            if (i < n) v[u] = NT ? __builtin_nontemporal_load(&src[i]) : src[i];
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const long long i = base + u * kStreamThreads + threadIdx.x;
            if (i < n) {
                if (NT) __builtin_nontemporal_store(v[u], &dst[i]);
                else dst[i] = v[u];
            }
        }
    }
}

}  // namespace
}  // namespace frkc2

using namespace frkc2;

extern "C" int frkc2_stream_copy(const void *src, void *dst, size_t bytes, int blocks_per_cu,
                                 int nontemporal, hipStream_t st)
{
    if (!src || !dst || bytes == 0 || (bytes & 15) || (((uintptr_t)src | (uintptr_t)dst) & 15) ||
        blocks_per_cu < 1 || blocks_per_cu > 64) {
        set_error("stream_copy: need 16-byte aligned non-NULL buffers, a multiple of 16 bytes "
                  "and 1 <= blocks_per_cu <= 64");
        return FRKC2_EINVAL;
    }
    int dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess || ncu < 1) {
        set_error("stream_copy: device query failed");
        return FRKC2_EHIP;
    }
    const long long n = (long long)(bytes / 16);
    long long blocks = (long long)ncu * blocks_per_cu;
    const long long need = (n + kStreamThreads * kUnroll - 1) / (kStreamThreads * kUnroll);
    if (blocks > need) blocks = need;
    if (nontemporal)
        hipLaunchKernelGGL(stream_copy<true>, dim3((unsigned)blocks), dim3(kStreamThreads), 0, st,
                           static_cast<const dvec2 *>(src), static_cast<dvec2 *>(dst), n);
    else
        hipLaunchKernelGGL(stream_copy<false>, dim3((unsigned)blocks), dim3(kStreamThreads), 0, st,
                           static_cast<const dvec2 *>(src), static_cast<dvec2 *>(dst), n);
    e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("stream_copy: HIP error %d (%s)", (int)e, hipGetErrorString(e));
        return FRKC2_EHIP;
    }
    return FRKC2_OK;
}
