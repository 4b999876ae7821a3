// copy.hip -- plain streaming device copy: the achievable-bandwidth reference
// for the sweep's roofline (the paper's data-transfer model, Sec. 4.1, has
// the memory-to-cache transfer dominate every pass; a copy moves exactly the
// bytes one pass must move, one read and one write per cell) and the known-
// size kernel that scales the FETCH_SIZE / WRITE_SIZE counters.
#include "dev_common.h"

namespace st {

// Each lane moves kU 16-byte vectors per iteration (all loads issued before
// the stores); work-groups stride over the buffer.
constexpr int kU = 4;

__global__ __launch_bounds__(256) void copy_kernel(const void* src, void* dst, int64_t nvec) {
    const ST_GLOBAL u32x4* s = gptr<u32x4>(src);
    ST_GLOBAL u32x4* d = gptr_mut<u32x4>(dst);
    const int64_t stride = static_cast<int64_t>(gridDim.x) * 256 * kU;
    for (int64_t base = static_cast<int64_t>(blockIdx.x) * 256 * kU + threadIdx.x; base < nvec; base += stride) {
        u32x4 v[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int64_t i = base + static_cast<int64_t>(u) * 256;
            if (i < nvec) v[u] = __builtin_nontemporal_load(s + i);
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int64_t i = base + static_cast<int64_t>(u) * 256;
            if (i < nvec) __builtin_nontemporal_store(v[u], d + i);
        }
    }
}

__global__ __launch_bounds__(256) void copy_tail_kernel(const unsigned char* src, unsigned char* dst, int64_t begin,
                                                        int64_t bytes) {
    const int64_t i = begin + static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i < bytes) dst[i] = src[i];
}

hipError_t launch_copy(void* dst, const void* src, int64_t bytes, int cus, hipStream_t s) {
    const int64_t nvec = bytes / 16;
    if (nvec > 0) {
        int64_t blocks = (nvec + 256 * kU - 1) / (256 * kU);
        const int64_t cap = static_cast<int64_t>(cus) * 8;  // eight work-groups per CU
        if (blocks > cap) blocks = cap;
        hipLaunchKernelGGL(copy_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, src, dst, nvec);
    }
    const int64_t done = nvec * 16;
    if (done < bytes) {
        const int64_t rest = bytes - done;
        hipLaunchKernelGGL(copy_tail_kernel, dim3(static_cast<unsigned>((rest + 255) / 256)), dim3(256), 0, s,
                           static_cast<const unsigned char*>(src), static_cast<unsigned char*>(dst), done, bytes);
    }
    return hipGetLastError();
}

}  // namespace st
