// varcoef.hip -- variable-coefficient 3D heat step and its adjoint.
//
// The paper's sweep has constant weights; differentiating a simulation with
// respect to a conductivity field needs the conservative variable form
// (zero-Dirichlet ghost layer, faces visited z-, z+, y-, y+, x-, x+):
//   u'[i] = u[i] + alpha * sum_f kap_f * (u[i+f] - u[i]),
//   kap_f = (k[i] + k[i+f]) / 2 inside the grid; kap_f = k[i], u = 0 on the
//   ghost layer.
// The step is a symmetric linear map of u, so its transpose is the same
// step applied to lambda.  The derivative of L through one step with respect
// to k, gathered per cell j (lambda = dL/du' , u = the state the step read):
//   dL/dk[j] += alpha * ( sum over inner faces f of j of
//                          (u[j+f] - u[j]) * (lambda[j] - lambda[j+f]) / 2
//                         - (number of ghost faces of j) * u[j] * lambda[j] ).
// (An inner face couples j and j+f: the term 0.5*(u_f-u_j) arises once from
// the update of j and once, with the opposite sign of the lambda difference,
// from the update of j+f; a ghost face contributes d kap/d k[j] = 1.)
// Both kernels are one thread per cell; a work-group covers 256 consecutive
// cells of one row (its row and plane come from the work-group index with
// 32-bit scalar arithmetic, so no lane divides), neighbours come through
// L1/L2, and work-groups are renumbered so each XCD streams a contiguous range
// of planes.
#include "dev_common.h"

namespace st {

// Unsigned 32-bit division by a divisor d fixed per launch, with the
// multiplier m = floor(2^32 (2^l - d) / d) + 1, l = ceil(log2 d) (the
// round-up method of Granlund and Montgomery, exact for every 32-bit n).
__device__ __forceinline__ uint32_t fdiv(uint32_t n, uint32_t m, uint32_t l) {
    if (l == 0) return n;
    const uint32_t t = __umulhi(m, n);
    return (t + ((n - t) >> 1)) >> (l - 1);
}
static void fdiv_init(uint32_t d, uint32_t& m, uint32_t& l) {
    l = 0;
    while ((uint64_t(1) << l) < d) ++l;
    m = l == 0 ? 0u : static_cast<uint32_t>(((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1);
}

// Work-group b (after the XCD renumbering) covers cells xb*256 .. +255 of
// row y of plane z, with b = (z*ny + y)*nxb + xb.
__device__ __forceinline__ bool cell_of(const VarcoefArgs& a, int64_t& x, int64_t& y, int64_t& z) {
    const uint32_t b = static_cast<uint32_t>(xcd_remap(blockIdx.x, gridDim.x));
    const uint32_t row = fdiv(b, a.nxb_m, a.nxb_l);
    const uint32_t zz = fdiv(row, a.ny_m, a.ny_l);
    x = static_cast<int64_t>(b - row * a.nxb) * 256 + threadIdx.x;
    y = row - zz * static_cast<uint32_t>(a.ny);
    z = zz;
    return x < a.nx;
}

template <typename TS>
__global__ __launch_bounds__(256) void varcoef_step_kernel(const VarcoefArgs a) {
    using TC = typename Storage<TS>::TC;
    const ST_GLOBAL TS* u = gptr<TS>(a.u);
    const ST_GLOBAL TS* k = gptr<TS>(a.k);
    ST_GLOBAL TS* out = gptr_mut<TS>(a.out);
    const int64_t nz = a.nz, ny = a.ny, nx = a.nx;
    int64_t x, y, z;
    if (!cell_of(a, x, y, z)) return;
    const int64_t i = (z * ny + y) * nx + x;
    const TC uc = ld1(u + i), kc = ld1(k + i);
    const TC alpha = static_cast<TC>(a.alpha);
    const int64_t dz[6] = {-1, 1, 0, 0, 0, 0}, dy[6] = {0, 0, -1, 1, 0, 0}, dx[6] = {0, 0, 0, 0, -1, 1};
    TC acc = TC(0);
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const int64_t zz = z + dz[f], yy = y + dy[f], xx = x + dx[f];
        if (zz >= 0 && zz < nz && yy >= 0 && yy < ny && xx >= 0 && xx < nx) {
            const int64_t j = (zz * ny + yy) * nx + xx;
            const TC kap = TC(0.5) * (kc + ld1(k + j));
            acc = fma_c(kap, ld1(u + j) - uc, acc);
        } else {
            acc = fma_c(kc, -uc, acc);
        }
    }
    st1(out + i, fma_c(alpha, acc, uc));
}

template <typename TS>
__global__ __launch_bounds__(256) void varcoef_adjoint_kernel(const VarcoefArgs a) {
    using TC = typename Storage<TS>::TC;
    const ST_GLOBAL TS* u = gptr<TS>(a.u);
    const ST_GLOBAL TS* k = gptr<TS>(a.k);
    const ST_GLOBAL TS* lam = gptr<TS>(a.lam);
    ST_GLOBAL TS* out = gptr_mut<TS>(a.out);
    ST_GLOBAL TS* g = gptr_mut<TS>(a.grad);
    const int64_t nz = a.nz, ny = a.ny, nx = a.nx;
    int64_t x, y, z;
    if (!cell_of(a, x, y, z)) return;
    const int64_t i = (z * ny + y) * nx + x;
    const TC uc = ld1(u + i), kc = ld1(k + i), lc = ld1(lam + i);
    const TC alpha = static_cast<TC>(a.alpha);
    const int64_t dz[6] = {-1, 1, 0, 0, 0, 0}, dy[6] = {0, 0, -1, 1, 0, 0}, dx[6] = {0, 0, 0, 0, -1, 1};
    TC acc = TC(0), gacc = TC(0);
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const int64_t zz = z + dz[f], yy = y + dy[f], xx = x + dx[f];
        if (zz >= 0 && zz < nz && yy >= 0 && yy < ny && xx >= 0 && xx < nx) {
            const int64_t j = (zz * ny + yy) * nx + xx;
            const TC kap = TC(0.5) * (kc + ld1(k + j));
            const TC lf = ld1(lam + j);
            acc = fma_c(kap, lf - lc, acc);
            gacc = fma_c(TC(0.5) * (ld1(u + j) - uc), lc - lf, gacc);
        } else {
            acc = fma_c(kc, -lc, acc);
            gacc = fma_c(-uc, lc, gacc);
        }
    }
    st1(out + i, fma_c(alpha, acc, lc));
    if (a.grad != nullptr) st1(g + i, fma_c(alpha, gacc, ld1(g + i)));
}

hipError_t launch_varcoef(int dtype, bool adjoint, const VarcoefArgs& args, hipStream_t s) {
    const int64_t blocks = args.nz * args.ny * ((args.nx + 255) / 256);
    if (blocks <= 0) return hipSuccess;
    if (blocks >= (int64_t(1) << 31)) return hipErrorInvalidValue;
    VarcoefArgs a = args;
    a.nxb = static_cast<uint32_t>((a.nx + 255) / 256);
    fdiv_init(a.nxb, a.nxb_m, a.nxb_l);
    fdiv_init(static_cast<uint32_t>(a.ny), a.ny_m, a.ny_l);
    const dim3 grid(static_cast<unsigned>(blocks)), block(256);
    if (dtype == kF64) {
        if (adjoint) hipLaunchKernelGGL(varcoef_adjoint_kernel<double>, grid, block, 0, s, a);
        else hipLaunchKernelGGL(varcoef_step_kernel<double>, grid, block, 0, s, a);
    } else if (dtype == kF32) {
        if (adjoint) hipLaunchKernelGGL(varcoef_adjoint_kernel<float>, grid, block, 0, s, a);
        else hipLaunchKernelGGL(varcoef_step_kernel<float>, grid, block, 0, s, a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace st
