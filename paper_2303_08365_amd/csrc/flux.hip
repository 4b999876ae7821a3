// flux.hip -- heat carried out of the grid across the zero-rule boundary.
//
// Reading the ghost layer of Alg. 1 (paper Sec. 2.1, Eq. 3) as an absorbing
// boundary: a step moves w_p * u(c) from cell c to the cell c - off_p that
// reads c through point p; whatever would land outside the grid has left.
// The leaving weight of a cell, sum_p w_p [c - off_p outside], is nonzero
// only within the pattern's reach of a face, so one step's outflow is a sum
// over that band of the state the step reads.
//
// Kernels:
//   * flux_band_kernel: the band sum of one state, per work-group, for any
//     point list (used when the steps run one per pass);
//   * flux_reduce_kernel: adds the per-work-group (or per-wave) partial sums
//     of one pass to the FP64 accumulator, in a fixed order, so the result
//     does not depend on scheduling;
//   * flux_reduce_batch_kernel: the same per grid of a batch pass, each grid's
//     work items being a contiguous range of the partial sums.
#include "dev_common.h"

namespace st {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ double block_sum(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if (static_cast<int>(threadIdx.x) < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    return red[0];
}

template <typename TS>
__global__ __launch_bounds__(kBlock) void flux_band_kernel(const FluxBandArgs a, double* part) {
    __shared__ double red[kBlock];
    const ST_GLOBAL TS* src = gptr<TS>(a.src);
    const int64_t nz = a.n[0], ny = a.n[1], nx = a.n[2];
    const int64_t rows = nz * ny;
    const int32_t rz = a.reach[0], ry = a.reach[1], rx = a.reach[2];
    const bool thin_x = nx <= 2 * static_cast<int64_t>(rx);
    double acc = 0.0;
    // a work-group per row: every cell of a row in the z or y band, the rx
    // cells at each end of the others
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const int64_t z = r / ny, y = r - z * ny;
        const bool full = thin_x || z < rz || z >= nz - rz || y < ry || y >= ny - ry;
        const int64_t cnt = full ? nx : 2 * static_cast<int64_t>(rx);
        for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x) {
            const int64_t x = full ? i : (i < rx ? i : nx - 2 * rx + i);
            double c = 0.0;
            for (int p = 0; p < a.npoints; ++p) {
                const int64_t tz = z - a.off[p][0], ty = y - a.off[p][1], tx = x - a.off[p][2];
                if (tz < 0 || tz >= nz || ty < 0 || ty >= ny || tx < 0 || tx >= nx) c += a.w[p];
            }
            if (c != 0.0) acc = fma(static_cast<double>(ld1(src + r * nx + x)), c, acc);
        }
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void flux_reduce_kernel(const double* part, int64_t n, double* flux) {
    __shared__ double red[kBlock];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kBlock) acc += part[i];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) flux[0] += s;
}

__global__ __launch_bounds__(kBlock) void flux_reduce_batch_kernel(const Stream2DGrid* table, const double* part,
                                                                     double* flux) {
    __shared__ double red[kBlock];
    const Stream2DGrid& d = table[blockIdx.x];
    const int64_t begin = d.tile_begin, n = d.items;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kBlock) acc += part[begin + i];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) flux[d.gid] += s;
}

}  // namespace

hipError_t launch_flux_reduce_batch(const Stream2DGrid* table, int count, const double* part, double* flux,
                                    hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(flux_reduce_batch_kernel, dim3(static_cast<unsigned>(count)), dim3(kBlock), 0, s, table, part,
                       flux);
    return hipGetLastError();
}

hipError_t launch_flux_band(int dtype, const FluxBandArgs& a, double* part, int nblocks, hipStream_t s) {
    if (nblocks < 1) return hipErrorInvalidValue;
    const dim3 grid(static_cast<unsigned>(nblocks)), block(kBlock);
    switch (dtype) {
        case kF64: hipLaunchKernelGGL(flux_band_kernel<double>, grid, block, 0, s, a, part); break;
        case kF32: hipLaunchKernelGGL(flux_band_kernel<float>, grid, block, 0, s, a, part); break;
        case kBF16: hipLaunchKernelGGL(flux_band_kernel<bf16s>, grid, block, 0, s, a, part); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_flux_reduce(const double* part, int64_t n, double* flux, hipStream_t s) {
    hipLaunchKernelGGL(flux_reduce_kernel, dim3(1), dim3(kBlock), 0, s, part, n, flux);
    return hipGetLastError();
}

}  // namespace st
