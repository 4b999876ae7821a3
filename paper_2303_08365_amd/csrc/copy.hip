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

// Stream-ordered upload of a small host table: each launch carries up to
// kTableWords 32-bit words in its argument block, so the runtime copies them
// when the launch is enqueued (or recorded into a graph) and the caller's
// host buffer is free at once -- no pinned staging buffer, no event to wait
// for, and a captured graph keeps its own copy of the table.
constexpr int kTableWords = 512;
struct TableChunk {
    uint32_t words[kTableWords];
};

__global__ __launch_bounds__(256) void table_write_kernel(uint32_t* dst, uint32_t nwords, const TableChunk c) {
    for (uint32_t i = threadIdx.x; i < nwords; i += 256) dst[i] = c.words[i];
}

hipError_t launch_table_write(void* dst, const void* src, size_t bytes, hipStream_t s) {
    if ((bytes & 3u) != 0 || (reinterpret_cast<uintptr_t>(dst) & 3u) != 0) return hipErrorInvalidValue;
    const size_t words = bytes / 4;
    const unsigned char* from = static_cast<const unsigned char*>(src);
    for (size_t w0 = 0; w0 < words; w0 += kTableWords) {
        const size_t n = words - w0 < static_cast<size_t>(kTableWords) ? words - w0 : kTableWords;
        TableChunk c;
        __builtin_memcpy(c.words, from + 4 * w0, 4 * n);
        hipLaunchKernelGGL(table_write_kernel, dim3(1), dim3(256), 0, s, static_cast<uint32_t*>(dst) + w0,
                           static_cast<uint32_t>(n), c);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace st
