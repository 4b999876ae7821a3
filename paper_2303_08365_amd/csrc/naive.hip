// naive.hip -- one time step per launch for any point list (ndim 1..3,
// radius <= 4, up to 125 points), one thread per cell.  This is the plain
// form of the sweep (paper Sec. 2.1, Alg. 1: every cell becomes the weighted
// sum of its pattern neighbours from the previous step) and the bitwise
// reference for the fused kernels: it evaluates the canonical point order
// with the same multiply / fma chain and the same ghost-cell zeros.
#include "dev_common.h"

namespace st {

template <typename TS>
__global__ __launch_bounds__(256) void naive_kernel(const NaiveArgs a) {
    using S = Storage<TS>;
    using TC = typename S::TC;
    const ST_GLOBAL TS* src = gptr<TS>(a.src);
    ST_GLOBAL TS* dst = gptr_mut<TS>(a.dst);
    const int64_t nz = a.n[0], ny = a.n[1], nx = a.n[2];
    const int64_t cells = nz * ny * nx;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < cells;
         i += stride) {
        const int64_t x = i % nx;
        const int64_t y = (i / nx) % ny;
        const int64_t z = i / (nx * ny);
        TC acc = TC(0);
        for (int p = 0; p < a.npoints; ++p) {
            int64_t zz = z + a.off[p][0], yy = y + a.off[p][1], xx = x + a.off[p][2];
            TC v = TC(0);
            const bool out = zz < 0 || zz >= nz || yy < 0 || yy >= ny || xx < 0 || xx >= nx;
            if (a.bc == kPeriodic) {
                zz = wrap_idx(zz, nz);
                yy = wrap_idx(yy, ny);
                xx = wrap_idx(xx, nx);
                v = ld1(src + (zz * ny + yy) * nx + xx);
            } else if (!out) {
                v = ld1(src + (zz * ny + yy) * nx + xx);
            }
            const TC w = static_cast<TC>(a.w[p]);
            acc = (p == 0) ? w * v : fma_c(w, v, acc);
        }
        st1(dst + i, acc);
    }
}

hipError_t launch_naive(int dtype, const NaiveArgs& a, hipStream_t s) {
    const int64_t cells = a.n[0] * a.n[1] * a.n[2];
    int64_t blocks = (cells + 255) / 256;
    if (blocks > (int64_t(1) << 20)) blocks = int64_t(1) << 20;
    if (blocks < 1) blocks = 1;
    const dim3 grid(static_cast<unsigned>(blocks)), block(256);
    switch (dtype) {
        case kF64: hipLaunchKernelGGL(naive_kernel<double>, grid, block, 0, s, a); break;
        case kF32: hipLaunchKernelGGL(naive_kernel<float>, grid, block, 0, s, a); break;
        case kBF16: hipLaunchKernelGGL(naive_kernel<bf16s>, grid, block, 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace st
