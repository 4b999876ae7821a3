// stream2d_impl.h -- 2D star/box stencils with T_b time steps fused per pass.
//
// Blocking in space and time (paper Sec. 4: tiles are held on chip and
// advanced several steps before they return to memory, Sec. 4.1; the GPU
// keeps global accesses coalesced through its on-chip staging, Sec. 4.2).
// The register-level mapping (Sec. 3: every neighbour is brought into the
// same slot as its centre without a trip through memory) is done here with
// wavefront DPP shifts instead of the paper's AVX2 swizzles or tensor-core
// folding.
//
// Work decomposition.  A wave owns an x strip of W = 64*VX columns: lane L
// holds columns X0 + L*VX .. X0 + L*VX + VX-1 of every row it touches, loaded
// with one coalesced 16-byte access per lane.  The wave walks the rows of one
// y chunk from top to bottom.  Pipeline level l (l = 0 .. tb-1) keeps the
// last 2R+1 rows of step l in registers; each new row of step l lets level
// l+1 produce the row R above it, so step tb leaves the wave R*tb rows behind
// the loads and is stored straight away.  x neighbours come from the lane's
// own registers or, across the lane boundary, from lane +-1 by DPP; y
// neighbours are other queue slots; nothing goes through LDS.
//
// Halo.  Step l is exact on columns [X0 - R + l*R, X0 + W + R - l*R); the
// outermost R columns of step 0 (outside the register strip) are loaded by
// lanes 0 and 63 and enter through the DPP "old" operand.  Only the strip
// interior [X0 + hxa, X0 + W - hxa), hxa >= R*(tb-1), is stored; strips
// overlap by 2*hxa columns.  Rows: a chunk of output rows [ys, ye) loads
// rows ys - R*tb .. ye - 1 + R*tb.
//
// Boundary.  Zero rule: cells outside the grid are forced to 0 at every
// step (they are ghost cells); periodic rule: loads wrap and the halo cells
// are genuine copies.
#pragma once

#include <utility>

#include "dev_common.h"
#include "registry.h"

namespace st {

namespace s2d {

template <typename TS, int R, int CLS, int TBMAX, int VX, bool PER>
struct Kern {
    using S = Storage<TS>;
    using TC = typename S::TC;
    static constexpr int Q = 2 * R + 1;  // rows per queue
    static constexpr int W = 64 * VX;     // register strip width
    static constexpr int NP = (CLS == kStar) ? 4 * R + 1 : Q * Q;

    struct Ctx {
        const TS* src;
        TS* dst;
        int64_t ny, nx;
        int64_t X0;       // first register column of the strip
        int64_t xl;       // first column of this lane
        int64_t ys, ye;   // output rows of the chunk
        int64_t ofirst, olast;  // output columns [ofirst, olast)
        bool fast;        // strip + ring inside the grid and aligned
        int lane;
        TC w[NP];
    };

    // Load row y of the input (step 0) for this lane, plus the ring values
    // held by the edge lanes.
    static __device__ __forceinline__ void load_row(const Ctx& c, int64_t y, TC (&v)[VX],
                                                    TC (&ext)[R]) {
        const bool yin = (y >= 0 && y < c.ny);
        if (!PER && !yin) {
#pragma unroll
            for (int e = 0; e < VX; ++e) v[e] = TC(0);
#pragma unroll
            for (int k = 0; k < R; ++k) ext[k] = TC(0);
            return;
        }
        const int64_t yy = PER ? wrap_idx(y, c.ny) : y;
        const TS* row = c.src + yy * c.nx;
        if (c.fast) {
            ldv<TS, VX>(row + c.xl, v);
        } else {
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                int64_t x = c.xl + e;
                if (PER) {
                    v[e] = ld1(row + wrap_idx(x, c.nx));
                } else {
                    v[e] = (x >= 0 && x < c.nx) ? ld1(row + x) : TC(0);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < R; ++k) ext[k] = TC(0);
        if (c.lane == 0 || c.lane == 63) {
            const int64_t xb = (c.lane == 0) ? c.X0 - R : c.X0 + W;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                int64_t x = xb + k;
                if (PER) {
                    ext[k] = ld1(row + wrap_idx(x, c.nx));
                } else {
                    ext[k] = (x >= 0 && x < c.nx) ? ld1(row + x) : TC(0);
                }
            }
        }
    }

    // Neighbours across the lane boundary of one row: lft[k] is column
    // xl - R + k (from lane-1), rgt[k] is column xl + VX + k (from lane+1).
    static __device__ __forceinline__ void side(const TC (&v)[VX], const TC (&ext)[R],
                                                TC (&lft)[R], TC (&rgt)[R]) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            lft[k] = from_lower(v[VX - R + k], ext[k]);
            rgt[k] = from_upper(v[k], ext[k]);
        }
    }

    static __device__ __forceinline__ TC xval(const TC (&v)[VX], const TC (&lft)[R],
                                              const TC (&rgt)[R], int idx) {
        // idx in [-R, VX + R): compile-time after unrolling
        return idx < 0 ? lft[R + idx] : (idx >= VX ? rgt[idx - VX] : v[idx]);
    }

    // One output row of step l+1 from the queue of step l.  J is the slot of
    // the newest row; slot of the row dy away from the centre is
    // (J - R + dy) mod Q.
    template <int J>
    static __device__ __forceinline__ void compute(const Ctx& c, const TC (&q)[Q][VX],
                                                   const TC (&ext)[Q][R], TC (&out)[VX]) {
        constexpr int CEN = (J - R + Q) % Q;
        if constexpr (CLS == kStar) {
            TC lft[R], rgt[R];
            side(q[CEN], ext[CEN], lft, rgt);
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                TC acc = c.w[0] * q[CEN][e];
                int p = 1;
#pragma unroll
                for (int dy = -R; dy <= -1; ++dy, ++p)
                    acc = fma_c(c.w[p], q[(J - R + dy + 2 * Q) % Q][e], acc);
#pragma unroll
                for (int dx = -R; dx <= -1; ++dx, ++p)
                    acc = fma_c(c.w[p], xval(q[CEN], lft, rgt, e + dx), acc);
#pragma unroll
                for (int dx = 1; dx <= R; ++dx, ++p)
                    acc = fma_c(c.w[p], xval(q[CEN], lft, rgt, e + dx), acc);
#pragma unroll
                for (int dy = 1; dy <= R; ++dy, ++p)
                    acc = fma_c(c.w[p], q[(J - R + dy + 2 * Q) % Q][e], acc);
                out[e] = acc;
            }
        } else {
            TC lft[Q][R], rgt[Q][R];
#pragma unroll
            for (int s = 0; s < Q; ++s) side(q[s], ext[s], lft[s], rgt[s]);
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                TC acc = c.w[0] * q[CEN][e];
                int p = 1;
#pragma unroll
                for (int dy = -R; dy <= R; ++dy) {
                    const int sl = (J - R + dy + 2 * Q) % Q;
#pragma unroll
                    for (int dx = -R; dx <= R; ++dx) {
                        if (dy == 0 && dx == 0) continue;
                        acc = fma_c(c.w[p], xval(q[sl], lft[sl], rgt[sl], e + dx), acc);
                        ++p;
                    }
                }
                out[e] = acc;
            }
        }
    }

    // Zero rule: a row or column outside the grid is a ghost and stays 0;
    // bfloat16 storage rounds every step's value.
    static __device__ __forceinline__ void finish(const Ctx& c, int64_t y, TC (&out)[VX]) {
        if (!PER) {
            if (y < 0 || y >= c.ny) {
#pragma unroll
                for (int e = 0; e < VX; ++e) out[e] = TC(0);
            } else if (!c.fast) {
#pragma unroll
                for (int e = 0; e < VX; ++e) {
                    const int64_t x = c.xl + e;
                    if (x < 0 || x >= c.nx) out[e] = TC(0);
                }
            }
        }
#pragma unroll
        for (int e = 0; e < VX; ++e) out[e] = S::round(out[e]);
    }

    static __device__ __forceinline__ void store_row(const Ctx& c, int64_t y, const TC (&out)[VX]) {
        if (y < c.ys || y >= c.ye) return;
        if (c.xl < c.ofirst || c.xl >= c.olast) return;  // lanes are wholly in or out
        TS* row = c.dst + y * c.nx;
        if (c.fast) {
            stv<TS, VX>(row + c.xl, out);
        } else {
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                const int64_t x = c.xl + e;
                if (x < c.nx) st1(row + x, out[e]);
            }
        }
    }

    template <int J>
    static __device__ __forceinline__ void step(const Ctx& c, int tb, int64_t it, int64_t nit,
                                                int64_t yfirst, TC (&pf)[Q][VX],
                                                TC (&pfx)[Q][R], TC (&q)[TBMAX][Q][VX],
                                                TC (&ext)[Q][R]) {
        const int64_t yin = yfirst + it;
        // step-0 row yin arrives from the prefetch slot; refill it Q rows ahead
#pragma unroll
        for (int e = 0; e < VX; ++e) q[0][J][e] = pf[J][e];
#pragma unroll
        for (int k = 0; k < R; ++k) ext[J][k] = pfx[J][k];
        if (it + Q < nit) load_row(c, yin + Q, pf[J], pfx[J]);
#pragma unroll
        for (int l = 0; l < TBMAX; ++l) {
            if (l < tb) {
                TC out[VX];
                if (l == 0) {
                    compute<J>(c, q[0], ext, out);
                } else {
                    TC zext[Q][R];
#pragma unroll
                    for (int s = 0; s < Q; ++s)
#pragma unroll
                        for (int k = 0; k < R; ++k) zext[s][k] = TC(0);
                    compute<J>(c, q[l], zext, out);
                }
                const int64_t yc = yin - static_cast<int64_t>(l + 1) * R;
                finish(c, yc, out);
                if (l + 1 == tb) {
                    store_row(c, yc, out);
                } else if (l + 1 < TBMAX) {
#pragma unroll
                    for (int e = 0; e < VX; ++e) q[l + 1][J][e] = out[e];
                }
            }
        }
    }

    static __device__ void run(const Stream2DArgs& a) {
        const int lane = threadIdx.x & 63;
        const int64_t wg = xcd_remap(blockIdx.x, gridDim.x);
        const int64_t item = __builtin_amdgcn_readfirstlane(static_cast<int>(wg * 4 + (threadIdx.x >> 6)));
        if (item >= a.items) return;
        const Stream2DGrid* gp = &a.one;
        if (a.grids != nullptr) {
            int lo = 0, hi = a.ngrids - 1;
            while (lo < hi) {  // last grid whose tile_begin <= item
                const int mid = (lo + hi + 1) >> 1;
                if (a.grids[mid].tile_begin <= item) lo = mid; else hi = mid - 1;
            }
            gp = a.grids + lo;
        }
        const int tb = gp->tb;
        Ctx c;
        c.src = static_cast<const TS*>(gp->src);
        c.dst = static_cast<TS*>(gp->dst);
        c.ny = gp->ny;
        c.nx = gp->nx;
        const int64_t local = item - gp->tile_begin;
        const int64_t tx = local % gp->tiles_x, cy = local / gp->tiles_x;
        c.X0 = tx * gp->out_w - gp->hxa;
        c.lane = lane;
        c.xl = c.X0 + static_cast<int64_t>(lane) * VX;
        c.ys = cy * gp->chunk_y;
        c.ye = c.ys + gp->chunk_y < c.ny ? c.ys + gp->chunk_y : c.ny;
        c.ofirst = c.X0 + gp->hxa;
        c.olast = c.ofirst + gp->out_w;
        c.fast = gp->vec_ok && (c.X0 - R >= 0) && (c.X0 + W + R <= c.nx);
#pragma unroll
        for (int p = 0; p < NP; ++p) c.w[p] = static_cast<TC>(gp->w[p]);

        const int64_t yfirst = c.ys - static_cast<int64_t>(R) * tb;
        const int64_t nit = (c.ye - c.ys) + 2 * static_cast<int64_t>(R) * tb;

        TC pf[Q][VX], pfx[Q][R], q[TBMAX][Q][VX], ext[Q][R];
#pragma unroll
        for (int l = 0; l < TBMAX; ++l)
#pragma unroll
            for (int s = 0; s < Q; ++s)
#pragma unroll
                for (int e = 0; e < VX; ++e) q[l][s][e] = TC(0);
#pragma unroll
        for (int s = 0; s < Q; ++s) {
#pragma unroll
            for (int k = 0; k < R; ++k) ext[s][k] = TC(0);
            if (s < nit) {
                load_row(c, yfirst + s, pf[s], pfx[s]);
            } else {
#pragma unroll
                for (int e = 0; e < VX; ++e) pf[s][e] = TC(0);
#pragma unroll
                for (int k = 0; k < R; ++k) pfx[s][k] = TC(0);
            }
        }
        for (int64_t base = 0; base < nit; base += Q) {
            unroll_steps(c, tb, base, nit, yfirst, pf, pfx, q, ext,
                         std::make_integer_sequence<int, Q>{});
        }
    }

    template <int... J>
    static __device__ __forceinline__ void unroll_steps(const Ctx& c, int tb, int64_t base,
                                                        int64_t nit, int64_t yfirst,
                                                        TC (&pf)[Q][VX], TC (&pfx)[Q][R],
                                                        TC (&q)[TBMAX][Q][VX], TC (&ext)[Q][R],
                                                        std::integer_sequence<int, J...>) {
        ((base + J < nit ? step<J>(c, tb, base + J, nit, yfirst, pf, pfx, q, ext) : void()), ...);
    }
};

template <typename TS, int R, int CLS, int TBMAX, int VX, bool PER>
__global__ __launch_bounds__(256) void stream2d_kernel(const Stream2DArgs a) {
    Kern<TS, R, CLS, TBMAX, VX, PER>::run(a);
}

template <typename TS, int R, int CLS, int TBMAX, int VX, bool PER>
void launch(const Stream2DArgs& a, hipStream_t s) {
    const int64_t wgs = (a.items + 3) / 4;
    hipLaunchKernelGGL((stream2d_kernel<TS, R, CLS, TBMAX, VX, PER>), dim3(static_cast<unsigned>(wgs)),
                       dim3(256), 0, s, a);
}

template <typename TS> constexpr int32_t dtype_of();
template <> constexpr int32_t dtype_of<double>() { return kF64; }
template <> constexpr int32_t dtype_of<float>() { return kF32; }
template <> constexpr int32_t dtype_of<bf16s>() { return kBF16; }

#define S2D_ENTRY(TS, R, CLS, TBM, VX, PER)                                                    \
    Entry2{Stream2DKey{dtype_of<TS>(), (PER) ? kPeriodic : kZero, CLS, R, TBM, VX},            \
           &launch<TS, R, CLS, TBM, VX, PER>}
#define S2D_BC(TS, R, CLS, TBM, VX) \
    S2D_ENTRY(TS, R, CLS, TBM, VX, false), S2D_ENTRY(TS, R, CLS, TBM, VX, true)

}  // namespace s2d
}  // namespace st
