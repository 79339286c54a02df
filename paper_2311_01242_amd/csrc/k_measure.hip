// Measurement helpers (not steps of the method): a plain device copy whose
// achieved bandwidth serves as the measured ceiling the gate kernels'
// rooflines are reported against, next to the vendor HBM peak, and an LDS
// read-modify-write loop for the on-chip side of the same kernels.  One launch
// copies `bytes` from src to dst `passes` times, so that a buffer pair small
// enough to stay in the last-level cache (MALL) is re-read from there, and a
// large one streams from HBM, with no launch gaps inside the timed region.
#include "device_common.h"

namespace vqe {

constexpr int kCopyThreads = 256;
constexpr int kCopyUnroll = 4;

__global__ void __launch_bounds__(kCopyThreads) k_copy_passes(const double2* __restrict__ src,
                                                              double2* __restrict__ dst, int64_t n,
                                                              int passes) {
    const int64_t stride = int64_t(gridDim.x) * kCopyThreads * kCopyUnroll;
    const int64_t first = int64_t(blockIdx.x) * kCopyThreads * kCopyUnroll + threadIdx.x;
    for (int p = 0; p < passes; ++p) {
        for (int64_t base = first; base < n; base += stride) {
            double2 v[kCopyUnroll];
#pragma unroll
            for (int u = 0; u < kCopyUnroll; ++u) {
                const int64_t k = base + int64_t(u) * kCopyThreads;
                if (k < n) v[u] = ldg2(src + k);
            }
#pragma unroll
            for (int u = 0; u < kCopyUnroll; ++u) {
                const int64_t k = base + int64_t(u) * kCopyThreads;
                if (k < n) stg2(dst + k, v[u]);
            }
        }
        // keep every pass: the compiler may not merge repeated loads/stores
        __asm__ volatile("" ::: "memory");
    }
}

// LDS ceiling: every thread reads eight 16-byte slots of its workgroup's
// 64 KiB array (consecutive lanes on consecutive slots: no bank conflicts),
// changes them and writes them back, iters times; the slots of one thread
// are its own, so no two threads touch one address.  Bytes moved = reads +
// writes.  The gate kernels move each pair's amplitudes through LDS the
// same way (read, rotate, write back).
constexpr int kLdsThreads = 512;
constexpr int kLdsSlots = 4096;   // double2 slots per workgroup (64 KiB)
constexpr int kLdsPerThread = kLdsSlots / kLdsThreads;

__global__ void __launch_bounds__(kLdsThreads) k_lds_rw(int iters, double* sink) {
    __shared__ double2 buf[kLdsSlots];
    for (int u = 0; u < kLdsPerThread; ++u)
        buf[threadIdx.x + u * kLdsThreads] = make_double2(double(threadIdx.x), 1.0);
    for (int it = 0; it < iters; ++it) {
        double2 v[kLdsPerThread];
#pragma unroll
        for (int u = 0; u < kLdsPerThread; ++u) v[u] = buf[threadIdx.x + u * kLdsThreads];
#pragma unroll
        for (int u = 0; u < kLdsPerThread; ++u) {
            v[u].y = v[u].y * 0.5 + v[u].x;
            buf[threadIdx.x + u * kLdsThreads] = v[u];
        }
        // every pass goes through LDS: no load or store may be kept in registers
        __asm__ volatile("" ::: "memory");
    }
    double acc = 0.0;
    for (int u = 0; u < kLdsPerThread; ++u) acc += buf[threadIdx.x + u * kLdsThreads].y;
    if (acc == -1.0) sink[0] = acc;   // never true (all values positive): keeps the loop
}

}  // namespace vqe

extern "C" int vqe_lds_ceiling(int iters, void* stream, double* ms, double* bytes) {
    using namespace vqe;
    if (!ms || !bytes) return fail(VQE_EINVAL, "null output");
    if (iters < 1 || iters > 1000000) return fail(VQE_ERANGE, "iters must be in [1, 1000000]");
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return fail(VQE_EDEVICE, "no HIP device");
    const int blocks = 2 * cus;   // two 64 KiB workgroups per CU
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail(VQE_EDEVICE, "hipEventCreate failed");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(VQE_EDEVICE, "hipEventCreate failed");
    }
    hipError_t err = hipEventRecord(e0, st);
    if (err == hipSuccess) {
        hipLaunchKernelGGL(k_lds_rw, dim3(blocks), dim3(kLdsThreads), 0, st, iters, nullptr);
        err = hipGetLastError();
    }
    if (err == hipSuccess) err = hipEventRecord(e1, st);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float t = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return fail(VQE_EDEVICE, std::string("LDS ceiling: ") + hipGetErrorString(err));
    *ms = double(t);
    *bytes = 2.0 * double(blocks) * kLdsSlots * sizeof(double2) * double(iters);
    return VQE_OK;
}

extern "C" int vqe_copy_ceiling(const void* src, void* dst, int64_t bytes, int passes, void* stream,
                                double* ms) {
    using namespace vqe;
    if (!src || !dst || !ms) return fail(VQE_EINVAL, "null buffer or output");
    if (bytes <= 0 || bytes % 16 != 0) return fail(VQE_ERANGE, "bytes must be a positive multiple of 16");
    if (passes < 1 || passes > 100000) return fail(VQE_ERANGE, "passes must be in [1, 100000]");
    if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15)
        return fail(VQE_EINVAL, "buffers must be 16-byte aligned");
    const int64_t n = bytes / 16;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return fail(VQE_EDEVICE, "no HIP device");
    const int64_t per_block = int64_t(kCopyThreads) * kCopyUnroll;
    const int64_t want = (n + per_block - 1) / per_block;
    const int blocks = int(std::min<int64_t>(want, int64_t(cus) * 8));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail(VQE_EDEVICE, "hipEventCreate failed");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(VQE_EDEVICE, "hipEventCreate failed");
    }
    hipError_t err = hipEventRecord(e0, st);
    if (err == hipSuccess) {
        hipLaunchKernelGGL(k_copy_passes, dim3(blocks), dim3(kCopyThreads), 0, st,
                           static_cast<const double2*>(src), static_cast<double2*>(dst), n, passes);
        err = hipGetLastError();
    }
    if (err == hipSuccess) err = hipEventRecord(e1, st);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float t = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return fail(VQE_EDEVICE, std::string("copy ceiling: ") + hipGetErrorString(err));
    *ms = double(t);
    return VQE_OK;
}
