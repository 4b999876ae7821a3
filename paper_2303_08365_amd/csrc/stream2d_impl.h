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
// neighbours are other queue slots; nothing goes through LDS.  The R columns
// just outside the strip (step 0 only) are fetched by lanes 0..R-1 (left) and
// 32..32+R-1 (right) with the row and reach the DPP "old" operand of lanes 0
// and 63 through readlane.
//
// Rows are prefetched 2R+1 rows ahead with unconditional loads (clamped or
// wrapped indices); ghost cells of the zero rule become 0 through selects
// when a row is consumed, so no branch separates a load from its use.
//
// Halo.  Step l is exact on columns [X0 - R + l*R, X0 + W + R - l*R); only
// the strip interior [X0 + hxa, X0 + W - hxa), hxa >= R*(tb-1), is stored.
// Under the zero rule a strip crossing the grid edge is moved inward to touch
// it (exact: the ghost layer is 0 at every step and lanes 0/63 receive 0).
// Rows: a chunk of output rows [ys, ye) streams rows ys - R*tb .. ye-1+R*tb.
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
    static_assert(VX >= R, "a lane must hold at least R columns");
    static constexpr int Q = 2 * R + 1;  // rows per queue, also the prefetch depth
    static constexpr int W = 64 * VX;     // register strip width
    static constexpr int NP = (CLS == kStar) ? 4 * R + 1 : Q * Q;

    struct Ctx {
        const ST_GLOBAL TS* src;
        ST_GLOBAL TS* dst;
        int64_t ny, nx;
        int64_t X0;             // first register column of the strip
        int64_t xl;             // first column of this lane
        int64_t xr_x;           // ring column this lane fetches
        int64_t ys, ye, ylast;  // output rows of the chunk; last streamed row
        int64_t ofirst, olast;  // output columns [ofirst, olast)
        int lane;
        TC w[NP];
    };

    static __device__ __forceinline__ int64_t fix(int64_t i, int64_t n) {
        if (PER) return wrap_idx(i, n);
        return i < 0 ? 0 : (i >= n ? n - 1 : i);
    }
    static __device__ __forceinline__ bool ghost(int64_t i, int64_t n) {
        return !PER && (i < 0 || i >= n);
    }

    template <bool FAST>
    static __device__ __forceinline__ void load_row(const Ctx& c, int64_t y, TC (&v)[VX], TC& xv) {
        const ST_GLOBAL TS* row = c.src + fix(y < c.ylast ? y : c.ylast, c.ny) * c.nx;
        if constexpr (FAST) {
            ldv<TS, VX>(row + (PER ? wrap_idx(c.xl, c.nx) : c.xl), v);
        } else {
#pragma unroll
            for (int e = 0; e < VX; ++e) v[e] = ld1(row + fix(c.xl + e, c.nx));
        }
        xv = ld1(row + fix(c.xr_x, c.nx));
    }

    template <bool FAST>
    static __device__ __forceinline__ void take_row(const Ctx& c, int64_t y, const TC (&v)[VX], TC xv,
                                                    TC (&out)[VX], TC& xo) {
        const bool yg = ghost(y, c.ny);
#pragma unroll
        for (int e = 0; e < VX; ++e) {
            const bool g = yg || (!FAST && ghost(c.xl + e, c.nx));
            out[e] = g ? TC(0) : v[e];
        }
        xo = (yg || ghost(c.xr_x, c.nx)) ? TC(0) : xv;
    }

    static __device__ __forceinline__ TC lane_value(TC v, int src_lane) {
        if constexpr (sizeof(TC) == 8) {
            const uint64_t b = __double_as_longlong(v);
            const uint32_t lo = __builtin_amdgcn_readlane(static_cast<int>(b), src_lane);
            const uint32_t hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), src_lane);
            return __longlong_as_double((static_cast<uint64_t>(hi) << 32) | lo);
        } else {
            return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src_lane));
        }
    }

    // Neighbours across the lane boundary of one row: lft[k] is column
    // xl - R + k (from lane-1), rgt[k] is column xl + VX + k (from lane+1).
    template <bool LEVEL0>
    static __device__ __forceinline__ void side(const TC (&v)[VX], TC xr, TC (&lft)[R], TC (&rgt)[R]) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const TC ol = LEVEL0 ? lane_value(xr, k) : TC(0);
            const TC orr = LEVEL0 ? lane_value(xr, 32 + k) : TC(0);
            lft[k] = from_lower(v[VX - R + k], ol);
            rgt[k] = from_upper(v[k], orr);
        }
    }

    static __device__ __forceinline__ TC xval(const TC (&v)[VX], const TC (&lft)[R],
                                              const TC (&rgt)[R], int idx) {
        return idx < 0 ? lft[R + idx] : (idx >= VX ? rgt[idx - VX] : v[idx]);
    }

    // One output row of step l+1 from the queue of step l.  J is the slot of
    // the newest row; the row dy away from the centre is slot (J - R + dy) mod
    // Q.  Canonical point order: centre, then (dy, dx) lexicographic.
    template <int J, bool LEVEL0>
    static __device__ __forceinline__ void compute(const Ctx& c, const TC (&q)[Q][VX], const TC (&xq)[Q],
                                                   TC (&out)[VX]) {
        constexpr int CEN = (J - R + Q) % Q;
        if constexpr (CLS == kStar) {
            TC lft[R], rgt[R];
            side<LEVEL0>(q[CEN], xq[CEN], lft, rgt);
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
            for (int s = 0; s < Q; ++s) side<LEVEL0>(q[s], xq[s], lft[s], rgt[s]);
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

    // Zero rule: ghost rows/columns stay 0; bfloat16 storage rounds every step.
    template <bool FAST>
    static __device__ __forceinline__ void finish(const Ctx& c, int64_t y, TC (&out)[VX]) {
        const bool yg = ghost(y, c.ny);
#pragma unroll
        for (int e = 0; e < VX; ++e) {
            const bool g = yg || (!FAST && ghost(c.xl + e, c.nx));
            out[e] = g ? TC(0) : S::round(out[e]);
        }
    }

    template <bool FAST>
    static __device__ __forceinline__ void store_row(const Ctx& c, int64_t y, const TC (&out)[VX]) {
        if (y < c.ys || y >= c.ye) return;
        if (c.xl < c.ofirst || c.xl >= c.olast) return;  // lanes are wholly in or out
        ST_GLOBAL TS* row = c.dst + y * c.nx;
        if constexpr (FAST) {
            stv<TS, VX>(row + c.xl, out);
        } else {
#pragma unroll
            for (int e = 0; e < VX; ++e)
                if (c.xl + e < c.nx) st1(row + c.xl + e, out[e]);
        }
    }

    struct State {
        TC q[TBMAX][Q][VX];
        TC xq[Q];           // step-0 ring values of the queued rows
        TC pf[Q][VX];
        TC pfx[Q];
    };

    template <bool FAST, int J>
    static __device__ __forceinline__ void step(const Ctx& c, int tb, int64_t it, int64_t yfirst, State& s) {
        const int64_t yin = yfirst + it;
        take_row<FAST>(c, yin, s.pf[J], s.pfx[J], s.q[0][J], s.xq[J]);
        load_row<FAST>(c, yin + Q, s.pf[J], s.pfx[J]);
#pragma unroll
        for (int l = 0; l < TBMAX; ++l) {
            if (l < tb) {
                TC out[VX];
                if (l == 0) {
                    compute<J, true>(c, s.q[0], s.xq, out);
                } else {
                    compute<J, false>(c, s.q[l], s.xq, out);
                }
                const int64_t yc = yin - static_cast<int64_t>(l + 1) * R;
                finish<FAST>(c, yc, out);
                if (l + 1 == tb) {
                    store_row<FAST>(c, yc, out);
                } else if (l + 1 < TBMAX) {
#pragma unroll
                    for (int e = 0; e < VX; ++e) s.q[l + 1][J][e] = out[e];
                }
            }
        }
    }

    template <bool FAST, int... J>
    static __device__ __forceinline__ void group(const Ctx& c, int tb, int64_t base, int64_t yfirst, State& s,
                                                 std::integer_sequence<int, J...>) {
        (step<FAST, J>(c, tb, base + J, yfirst, s), ...);
    }
    template <bool FAST, int... J>
    static __device__ __forceinline__ void tail(const Ctx& c, int tb, int64_t base, int64_t nit, int64_t yfirst,
                                                State& s, std::integer_sequence<int, J...>) {
        ((base + J < nit ? step<FAST, J>(c, tb, base + J, yfirst, s) : void()), ...);
    }

    template <bool FAST>
    static __device__ void body(Ctx& c, int tb) {
        const int64_t yfirst = c.ys - static_cast<int64_t>(R) * tb;
        const int64_t nit = (c.ye - c.ys) + 2 * static_cast<int64_t>(R) * tb;
        c.ylast = yfirst + nit - 1;
        State s;
#pragma unroll
        for (int l = 0; l < TBMAX; ++l)
#pragma unroll
            for (int sl = 0; sl < Q; ++sl)
#pragma unroll
                for (int e = 0; e < VX; ++e) s.q[l][sl][e] = TC(0);
#pragma unroll
        for (int sl = 0; sl < Q; ++sl) {
            s.xq[sl] = TC(0);
            load_row<FAST>(c, yfirst + sl, s.pf[sl], s.pfx[sl]);
        }
        int64_t base = 0;
        for (; base + Q <= nit; base += Q) group<FAST>(c, tb, base, yfirst, s, std::make_integer_sequence<int, Q>{});
        tail<FAST>(c, tb, base, nit, yfirst, s, std::make_integer_sequence<int, Q>{});
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
        // the descriptor may live in global memory: pin every field to SGPRs
        const int tb = uni(gp->tb);
        const int64_t tiles_x = uni(static_cast<int64_t>(gp->tiles_x));
        const int64_t out_w = uni(static_cast<int64_t>(gp->out_w));
        const int64_t hxa = uni(static_cast<int64_t>(gp->hxa));
        const int64_t chunk_y = uni(static_cast<int64_t>(gp->chunk_y));
        const bool vec_ok = uni(gp->vec_ok) != 0;
        Ctx c;
        c.src = gptr<TS>(uni(gp->src));
        c.dst = gptr_mut<TS>(uni(gp->dst));
        c.ny = uni(gp->ny);
        c.nx = uni(gp->nx);
        c.lane = lane;
        const int64_t local = item - uni(gp->tile_begin);
        const int64_t tx = local % tiles_x, cy = local / tiles_x;
        c.ofirst = tx * out_w;
        c.olast = c.ofirst + out_w < c.nx ? c.ofirst + out_w : c.nx;
        c.X0 = c.ofirst - hxa;
        const bool fast = vec_ok && (PER || c.nx >= W);
        if (!PER && fast) c.X0 = c.X0 < 0 ? 0 : (c.X0 + W > c.nx ? c.nx - W : c.X0);
        c.xl = c.X0 + static_cast<int64_t>(lane) * VX;
        {
            const bool right = lane >= 32;
            const int k = right ? lane - 32 : lane;
            c.xr_x = right && k < R ? c.X0 + W + k : c.X0 - R + (k < R ? k : 0);
        }
        c.ys = cy * chunk_y;
        c.ye = c.ys + chunk_y < c.ny ? c.ys + chunk_y : c.ny;
#pragma unroll
        for (int p = 0; p < NP; ++p) c.w[p] = static_cast<TC>(uni(gp->w[p]));
        if (fast) body<true>(c, tb);
        else body<false>(c, tb);
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

template <typename TS, int R, int CLS, int TBMAX, int VX, bool PER>
int occ_of() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, stream2d_kernel<TS, R, CLS, TBMAX, VX, PER>, 256, 0) !=
        hipSuccess)
        n = 0;
    return n;
}

template <typename TS> constexpr int32_t dtype_of();
template <> constexpr int32_t dtype_of<double>() { return kF64; }
template <> constexpr int32_t dtype_of<float>() { return kF32; }
template <> constexpr int32_t dtype_of<bf16s>() { return kBF16; }

#define S2D_ENTRY(TS, R, CLS, TBM, VX, PER)                                                    \
    Entry2{Stream2DKey{dtype_of<TS>(), (PER) ? kPeriodic : kZero, CLS, R, TBM, VX},            \
           &launch<TS, R, CLS, TBM, VX, PER>, &occ_of<TS, R, CLS, TBM, VX, PER>}
#define S2D_BC(TS, R, CLS, TBM, VX) \
    S2D_ENTRY(TS, R, CLS, TBM, VX, false), S2D_ENTRY(TS, R, CLS, TBM, VX, true)

}  // namespace s2d
}  // namespace st
