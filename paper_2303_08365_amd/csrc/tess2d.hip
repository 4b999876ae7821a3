// tess2d.hip -- 2D stars and boxes with the tessellated (non-redundant)
// temporal tiling along y: paper Sec. 4.1 tiles space-time with triangles,
// whose centre advances all T_b steps and whose cells near the edge fewer, and
// then with inverted triangles made of the halves of two neighbouring
// triangles, which bring every cell to T_b steps -- no cell is updated twice.
//
// On the GPU the triangles are the y chunks of the 2D streaming kernel run
// without halo rows (stage 1, stream2d_impl.h with TESS): a chunk's row at
// distance d from a junction (a boundary shared with the next chunk) is exact
// up to state L = min(T_b, d / R); rows with L = T_b are stored, and the two
// highest exact states of the others ("top" = state L, "pen" = state L - 1)
// go to the junction's band scratch.  Stage 2 (this file) is the inverted
// triangle: one wave per (junction, x strip) holds the 2R(T_b + 1) band rows
// around the junction in registers and brings them level by level to T_b:
// state t of a row with L < t is computed from the rows' states t - 1 (the
// same canonical multiply-FMA chain as every kernel, so the result is bit for
// bit the plain sweep's); a row with L = t takes its top, a row with L = t + 1
// its pen.  Every row's L is known at compile time (it depends only on its
// place in the band), so the schedule has no run-time tests.
//
// x keeps the overlapped strips of the streaming kernel: state 0 of a band
// row comes with its ring values (the R columns beyond each end of the
// strip), so the first step is exact on the whole strip and step t on all but
// (t - 1)R columns at each end, as in stage 1 (a halo of hxa >= R(T_b - 1)
// columns); deeper steps take zero through DPP at the strip's ends (under the
// zero rule strips at the grid's x edges move inward, where that zero is the
// ghost layer).
#include "stream2d_impl.h"

namespace st {
namespace s2d {

template <typename TS, int R, int CLS, int TB, int VX, bool PER>
struct Band {
    using S = Storage<TS>;
    using TC = typename S::TC;
    static constexpr int W = 64 * VX;
    static constexpr int NP = (CLS == kStar) ? 4 * R + 1 : (2 * R + 1) * (2 * R + 1);
    static constexpr int BR = tess_band_rows(R, TB);
    static constexpr int H = R * (TB + 1);  // band rows on each side of the junction
    static constexpr int32_t kRsrcWord3 = 0x00020000;
    static_assert(sizeof(TS) >= 4, "no per-step rounding: FP64 and FP32 storage only");

    // last exact state of band row b after stage 1
    static constexpr int level_of(int b) {
        const int d = b < H ? H - 1 - b : b - H;
        return d / R < TB ? d / R : TB;
    }

    using KK = Kern<TS, R, CLS, TB, VX, PER, false, true>;

    static __device__ __forceinline__ void ldrow(const TS* row, int lane, TC (&v)[VX]) {
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<TS*>(row), 0, static_cast<uint32_t>(W * sizeof(TS)), kRsrcWord3);
        KK::bloadv(r, static_cast<uint32_t>(lane * VX * sizeof(TS)), v);
    }

    // x neighbours across the lane boundary: the ring values at the strip's
    // ends for state 0 (RING), zero for deeper states
    template <bool RING>
    static __device__ __forceinline__ void side(const TC (&v)[VX], TC xr, TC (&lft)[R], TC (&rgt)[R]) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if constexpr (RING) {
                lft[k] = from_lower(v[VX - R + k], KK::lane_value(xr, k));
                rgt[k] = from_upper(v[k], KK::lane_value(xr, 32 + k));
            } else {
                lft[k] = from_lower_z(v[VX - R + k]);
                rgt[k] = from_upper_z(v[k]);
            }
        }
    }
    static __device__ __forceinline__ TC xval(const TC (&v)[VX], const TC (&lft)[R], const TC (&rgt)[R], int idx) {
        return idx < 0 ? lft[R + idx] : (idx >= VX ? rgt[idx - VX] : v[idx]);
    }

    // State t of band row b from the states t - 1 of rows b - R .. b + R,
    // canonical order: centre, then the star's y-, x-, x+, y+ points, or the
    // box's points with (dy, dx) lexicographic.
    template <int B, bool RING>
    static __device__ __forceinline__ void row_step(const TC (&w)[NP], const TC (&v)[BR][VX], const TC (&xr)[BR],
                                                    TC (&out)[VX]) {
        static_assert(B - R >= 0 && B + R < BR, "a computed row's neighbours lie in the band");
        if constexpr (CLS == kStar) {
            TC lft[R], rgt[R];
            side<RING>(v[B], xr[B], lft, rgt);
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                TC acc = w[0] * v[B][e];
                int p = 1;
#pragma unroll
                for (int dy = -R; dy <= -1; ++dy, ++p) acc = fma_c(w[p], v[B + dy][e], acc);
#pragma unroll
                for (int dx = -R; dx <= -1; ++dx, ++p) acc = fma_c(w[p], xval(v[B], lft, rgt, e + dx), acc);
#pragma unroll
                for (int dx = 1; dx <= R; ++dx, ++p) acc = fma_c(w[p], xval(v[B], lft, rgt, e + dx), acc);
#pragma unroll
                for (int dy = 1; dy <= R; ++dy, ++p) acc = fma_c(w[p], v[B + dy][e], acc);
                out[e] = acc;
            }
        } else {
            TC lft[2 * R + 1][R], rgt[2 * R + 1][R];
#pragma unroll
            for (int dy = -R; dy <= R; ++dy) side<RING>(v[B + dy], xr[B + dy], lft[dy + R], rgt[dy + R]);
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                TC acc = w[0] * v[B][e];
                int p = 1;
#pragma unroll
                for (int dy = -R; dy <= R; ++dy) {
#pragma unroll
                    for (int dx = -R; dx <= R; ++dx) {
                        if (dy == 0 && dx == 0) continue;
                        acc = fma_c(w[p], xval(v[B + dy], lft[dy + R], rgt[dy + R], e + dx), acc);
                        ++p;
                    }
                }
                out[e] = acc;
            }
        }
    }

    // Ghost columns (zero rule, element-wise strips that cross the grid's x
    // edge) stay 0 at every state.
    template <bool FAST>
    static __device__ __forceinline__ void clear_ghosts(int32_t xl, int32_t nx, TC (&v)[VX]) {
        if constexpr (!FAST && !PER) {
#pragma unroll
            for (int e = 0; e < VX; ++e) v[e] = static_cast<uint32_t>(xl + e) >= static_cast<uint32_t>(nx) ? TC(0) : v[e];
        }
    }

    // Level T: rows with L < T computed, rows with L = T take their top, rows
    // with L = T + 1 their pen.
    template <bool FAST, int T, int B = 0>
    static __device__ __forceinline__ void level_rows(const TC (&w)[NP], const TC (&v)[BR][VX], const TC (&xr)[BR],
                                                      TC (&nv)[BR][VX], const TS* top, const TS* pen, int lane,
                                                      int32_t xl, int32_t nx) {
        if constexpr (B < BR) {
            constexpr int L = level_of(B);
            if constexpr (L < T) {
                row_step<B, T == 1>(w, v, xr, nv[B]);
                clear_ghosts<FAST>(xl, nx, nv[B]);
            } else if constexpr (L == T && T < TB) {
                ldrow(top + B * W, lane, nv[B]);
            } else if constexpr (L == T + 1) {
                ldrow(pen + B * W, lane, nv[B]);
            } else {
#pragma unroll
                for (int e = 0; e < VX; ++e) nv[B][e] = v[B][e];
            }
            level_rows<FAST, T, B + 1>(w, v, xr, nv, top, pen, lane, xl, nx);
        }
    }
    template <bool FAST, int T = 1>
    static __device__ __forceinline__ void levels(const TC (&w)[NP], TC (&v)[BR][VX], const TC (&xr)[BR],
                                                  const TS* top, const TS* pen, int lane, int32_t xl, int32_t nx) {
        if constexpr (T <= TB) {
            TC nv[BR][VX];
            level_rows<FAST, T>(w, v, xr, nv, top, pen, lane, xl, nx);
#pragma unroll
            for (int b = 0; b < BR; ++b)
#pragma unroll
                for (int e = 0; e < VX; ++e) v[b][e] = nv[b][e];
            levels<FAST, T + 1>(w, v, xr, top, pen, lane, xl, nx);
        }
    }

    template <bool FAST>
    static __device__ __forceinline__ void body(const Stream2DGrid& g, const Stream2DArgs& a, int32_t j, int32_t tx,
                                                int lane) {
        const int32_t ny = static_cast<int32_t>(uni(g.ny)), nx = static_cast<int32_t>(uni(g.nx));
        const int32_t out_w = uni(g.out_w), hxa = uni(g.hxa), chunk_y = uni(g.chunk_y);
        const int32_t tiles_x = uni(g.tiles_x);
        const int32_t ofirst = tx * out_w;
        const int32_t olast = ofirst + out_w < nx ? ofirst + out_w : nx;
        int32_t X0 = ofirst - hxa;
        if (!PER && FAST) X0 = X0 < 0 ? 0 : (X0 + W > nx ? nx - W : X0);
        const int32_t xl = X0 + lane * VX;
        TC w[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) w[p] = static_cast<TC>(uni(g.w[p]));
        const TS* top =
            static_cast<const TS*>(a.tess) + (static_cast<int64_t>(j) * tiles_x + tx) * (BR * (2 * W + 64));
        const TS* pen = top + BR * W;
        const TS* ring = top + 2 * BR * W;
        // state 0 of the rows that need it (L = 0: top; L = 1: pen), with
        // its ring values
        TC v[BR][VX], xr[BR];
#pragma unroll
        for (int b = 0; b < BR; ++b) {
            if (level_of(b) <= 1) {
                ldrow((level_of(b) == 0 ? top : pen) + b * W, lane, v[b]);
                const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
                    const_cast<TS*>(ring + b * 64), 0, static_cast<uint32_t>(64 * sizeof(TS)), kRsrcWord3);
                xr[b] = KK::bload1(r, static_cast<uint32_t>(lane * sizeof(TS)));
            } else {
#pragma unroll
                for (int e = 0; e < VX; ++e) v[b][e] = TC(0);
                xr[b] = TC(0);
            }
        }
        levels<FAST>(w, v, xr, top, pen, lane, xl, nx);
        // the rows stage 1 did not finish: L < T_b
        TS* dst = static_cast<TS*>(uni(g.dst));
        const int32_t J = j * chunk_y;
        const uint32_t so = static_cast<uint32_t>(xl - ofirst) * sizeof(TS);
        const uint32_t out_bytes = static_cast<uint32_t>(olast - ofirst) * sizeof(TS);
#pragma unroll
        for (int b = 0; b < BR; ++b) {
            if (level_of(b) >= TB) continue;
            const int32_t y0 = J - H + b;
            const int32_t y = PER ? wrap_idx(y0, ny) : y0;
            TS* base = dst + static_cast<int64_t>(y) * nx + ofirst;
            const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(base, 0, out_bytes, kRsrcWord3);
            if constexpr (FAST) {
                KK::bstorev(r, so, v[b]);
            } else {
#pragma unroll
                for (int e = 0; e < VX; ++e) KK::bstore1(r, so + e * static_cast<uint32_t>(sizeof(TS)), v[b][e]);
            }
        }
    }

    static __device__ __forceinline__ void run(const Stream2DArgs& a) {
        const int lane = threadIdx.x & 63;
        const int64_t wg = xcd_remap(blockIdx.x, gridDim.x);
        const int64_t item = __builtin_amdgcn_readfirstlane(static_cast<int>(wg * 4 + (threadIdx.x >> 6)));
        const Stream2DGrid& g = a.one;
        const int32_t tiles_x = uni(g.tiles_x), chunks = uni(g.chunks_y);
        // junctions: zero rule 1 .. chunks - 1, periodic 0 .. chunks - 1
        const int32_t first = PER ? 0 : 1;
        const int64_t njunc = chunks - first;
        if (njunc <= 0 || item >= njunc * tiles_x) return;
        const int32_t j = static_cast<int32_t>(item / tiles_x) + first;
        const int32_t tx = static_cast<int32_t>(item % tiles_x);
        const bool vec_ok = uni(g.vec_ok) != 0;
        const bool fast = vec_ok && (PER || uni(g.nx) >= W);
        if (fast) body<true>(g, a, j, tx, lane);
        else body<false>(g, a, j, tx, lane);
    }
};

template <typename TS, int R, int CLS, int TB, int VX, bool PER>
__global__ __launch_bounds__(256) void tess2d_band_kernel(const Stream2DArgs a) {
    Band<TS, R, CLS, TB, VX, PER>::run(a);
}

template <typename TS, int R, int CLS, int TB, int VX, bool PER>
hipError_t band_launch(const Stream2DArgs& a, hipStream_t s) {
    const int64_t njunc = a.one.chunks_y - (PER ? 0 : 1);
    if (njunc <= 0) return hipSuccess;
    const int64_t items = njunc * a.one.tiles_x;
    hipLaunchKernelGGL((tess2d_band_kernel<TS, R, CLS, TB, VX, PER>), dim3(static_cast<unsigned>((items + 3) / 4)),
                       dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename TS, int R, int CLS, int VX, bool PER>
hipError_t band_tb(int tb, const Stream2DArgs& a, hipStream_t s) {
    switch (tb) {
        case 1: return band_launch<TS, R, CLS, 1, VX, PER>(a, s);
        case 2: return band_launch<TS, R, CLS, 2, VX, PER>(a, s);
        case 3: return band_launch<TS, R, CLS, 3, VX, PER>(a, s);
        case 4: return band_launch<TS, R, CLS, 4, VX, PER>(a, s);
        default: return hipErrorInvalidValue;
    }
}

// Stage-1 instances: FP64 and FP32, radius-1 and radius-2 stars and boxes,
// up to four fused steps, both boundary rules.
static const Entry2 kTessTable[] = {
    S2D_TESS(double, 1, kStar, 4, 2), S2D_TESS(double, 1, kBox, 4, 2), S2D_TESS(double, 2, kStar, 4, 2),
    S2D_TESS(double, 2, kBox, 4, 2),  S2D_TESS(float, 1, kStar, 4, 4), S2D_TESS(float, 1, kBox, 4, 4),
    S2D_TESS(float, 2, kStar, 4, 4),  S2D_TESS(float, 2, kBox, 4, 4),
};

}  // namespace s2d

Table2 s2d_table_tess() {
    return Table2{s2d::kTessTable, static_cast<int>(sizeof(s2d::kTessTable) / sizeof(s2d::kTessTable[0]))};
}

hipError_t launch_tess2d_band(const Stream2DKey& k, const Stream2DArgs& a, hipStream_t s) {
    const int tb = a.one.tb;
    const bool per = k.bc == kPeriodic;
#define ST_BAND(TS, R, CLS, VX)                                                                 \
    return per ? s2d::band_tb<TS, R, CLS, VX, true>(tb, a, s) : s2d::band_tb<TS, R, CLS, VX, false>(tb, a, s)
    if (k.dtype == kF64 && k.vx == 2) {
        if (k.radius == 1 && k.cls == kStar) ST_BAND(double, 1, kStar, 2);
        if (k.radius == 1 && k.cls == kBox) ST_BAND(double, 1, kBox, 2);
        if (k.radius == 2 && k.cls == kStar) ST_BAND(double, 2, kStar, 2);
        if (k.radius == 2 && k.cls == kBox) ST_BAND(double, 2, kBox, 2);
    }
    if (k.dtype == kF32 && k.vx == 4) {
        if (k.radius == 1 && k.cls == kStar) ST_BAND(float, 1, kStar, 4);
        if (k.radius == 1 && k.cls == kBox) ST_BAND(float, 1, kBox, 4);
        if (k.radius == 2 && k.cls == kStar) ST_BAND(float, 2, kStar, 4);
        if (k.radius == 2 && k.cls == kBox) ST_BAND(float, 2, kBox, 4);
    }
#undef ST_BAND
    return hipErrorInvalidValue;
}

}  // namespace st
