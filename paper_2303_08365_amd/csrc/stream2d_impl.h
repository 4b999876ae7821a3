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
// Loads.  Rows are prefetched 2R+1 rows ahead with buffer loads through a
// descriptor whose range is the row; under the zero rule a row outside the
// grid gets an empty range and a ghost column a 32-bit offset past the row's
// end, so ghost cells load as 0 -- no masks, no clamped indices, and no
// branch between a load and its use.  Lanes address their columns with a
// 32-bit offset fixed for the whole run.  Stores are buffer stores through a
// descriptor covering the strip's output columns of the row (empty for rows
// the chunk does not own), so every row issues the same stores.  The pipeline
// is specialised for the pass's depth (no run-time level tests in the loop).
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

template <typename TS, int R, int CLS, int TBMAX, int VX, bool PER, bool FLX, bool TESS = false>
struct Kern {
    using S = Storage<TS>;
    using TC = typename S::TC;
    static_assert(VX >= R, "a lane must hold at least R columns");
    static constexpr int Q = 2 * R + 1;  // rows per queue, also the prefetch depth
    static constexpr int W = 64 * VX;     // register strip width
    static constexpr int NP = (CLS == kStar) ? 4 * R + 1 : Q * Q;
    static constexpr int32_t kRsrcWord3 = 0x00020000;  // gfx9: raw 32-bit data
    static constexpr int32_t kNT = 2;                  // store cache policy: non-temporal

    struct Ctx {
        const TS* src;
        TS* dst;
        int32_t ny, nx;
        uint32_t row_bytes;
        int32_t X0;             // first register column of the strip
        int32_t xl;             // first column of this lane
        int32_t ys, ye, ylast;  // output rows of the chunk; last streamed row
        int32_t ylast_w;        // the last streamed row as loaded (wrapped)
        int32_t ofirst, olast;  // output columns [ofirst, olast)
        uint32_t lo;            // byte offset of this lane's first column
        uint32_t eo[VX];        // byte offsets of its columns (element access)
        uint32_t xr_off;        // byte offset of the ring column this lane fetches
        uint32_t so, out_bytes; // store: lane offset from ofirst, output row bytes
        int lane;
        TC w[NP];
        double* fpart;          // FLX: this wave's partial outflow slot
        bool fx;                // FLX: the strip owns a column within R of an x face
        bool fyb;               // FLX: the chunk owns a row within R of a y face
        // TESS: rows [cs, ce) of the chunk, a junction with the neighbouring
        // chunk above (jlo) / below (jhi); distances to a junction count
        // from clo (the chunk's first row) and chi (its last row), set far
        // away on a side without one; blo / bhi: this strip's band blocks
        // of the two junctions
        int32_t cs, ce;
        bool jlo, jhi;
        int32_t clo, chi;
        TS* blo;
        TS* bhi;
    };

    static __device__ __forceinline__ bool ghost(int32_t i, int32_t n) {
        return !PER && static_cast<uint32_t>(i) >= static_cast<uint32_t>(n);  // i < 0 or i >= n
    }

    static __device__ __forceinline__ TC bload1(__amdgpu_buffer_rsrc_t r, uint32_t off) {
        if constexpr (sizeof(TS) == 8) {
            return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
        } else if constexpr (sizeof(TS) == 4) {
            return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
        } else {
            return bf16_to_f32(__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0));
        }
    }
    static __device__ __forceinline__ void bloadv(__amdgpu_buffer_rsrc_t r, uint32_t off, TC (&v)[VX]) {
        constexpr int kBytes = VX * static_cast<int>(sizeof(TS));
        static_assert(kBytes % 8 == 0, "vector rows need whole 8-byte units");
        TS vals[VX];
        if constexpr (kBytes % 16 == 0) {
            u32x4 raw[kBytes / 16];
#pragma unroll
            for (int i = 0; i < kBytes / 16; ++i)
                raw[i] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(r, off + 16 * i, 0, 0));
            __builtin_memcpy(vals, raw, kBytes);
        } else {
            u32x2 raw[kBytes / 8];
#pragma unroll
            for (int i = 0; i < kBytes / 8; ++i)
                raw[i] = __builtin_bit_cast(u32x2, __builtin_amdgcn_raw_buffer_load_b64(r, off + 8 * i, 0, 0));
            __builtin_memcpy(vals, raw, kBytes);
        }
#pragma unroll
        for (int e = 0; e < VX; ++e) v[e] = S::widen(vals[e]);
    }
    static __device__ __forceinline__ void bstore1(__amdgpu_buffer_rsrc_t r, uint32_t off, TC v) {
        const TS x = S::narrow(v);
        if constexpr (sizeof(TS) == 8) {
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, off, 0, kNT);
        } else if constexpr (sizeof(TS) == 4) {
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, x), r, off, 0, kNT);
        } else {
            __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, x), r, off, 0, kNT);
        }
    }
    static __device__ __forceinline__ void bstorev(__amdgpu_buffer_rsrc_t r, uint32_t off, const TC (&v)[VX]) {
        constexpr int kBytes = VX * static_cast<int>(sizeof(TS));
        TS vals[VX];
#pragma unroll
        for (int e = 0; e < VX; ++e) vals[e] = S::narrow(v[e]);
        if constexpr (kBytes % 16 == 0) {
            u32x4 raw[kBytes / 16];
            __builtin_memcpy(raw, vals, kBytes);
#pragma unroll
            for (int i = 0; i < kBytes / 16; ++i) __builtin_amdgcn_raw_buffer_store_b128(raw[i], r, off + 16 * i, 0, kNT);
        } else {
            u32x2 raw[kBytes / 8];
            __builtin_memcpy(raw, vals, kBytes);
#pragma unroll
            for (int i = 0; i < kBytes / 8; ++i) __builtin_amdgcn_raw_buffer_store_b64(raw[i], r, off + 8 * i, 0, kNT);
        }
    }

    // Row y (wrapped already when periodic): an empty range outside the grid.
    template <bool FAST>
    static __device__ __forceinline__ void load_row(const Ctx& c, int32_t y, TC (&v)[VX], TC& xv) {
        const bool out = ghost(y, c.ny);
        const TS* base = out ? c.src : c.src + static_cast<int64_t>(y) * c.nx;
        const __amdgpu_buffer_rsrc_t r =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<TS*>(base), 0, out ? 0 : c.row_bytes, kRsrcWord3);
        if constexpr (FAST) {
            bloadv(r, c.lo, v);
        } else {
#pragma unroll
            for (int e = 0; e < VX; ++e) v[e] = bload1(r, c.eo[e]);
        }
        xv = bload1(r, c.xr_off);
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
    // Step 0 takes the strip's outer columns from the ring value; deeper steps
    // take 0 there (those columns are outside the exact region).
    template <bool LEVEL0>
    static __device__ __forceinline__ void side(const TC (&v)[VX], TC xr, TC (&lft)[R], TC (&rgt)[R]) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if constexpr (LEVEL0) {
                lft[k] = from_lower(v[VX - R + k], lane_value(xr, k));
                rgt[k] = from_upper(v[k], lane_value(xr, 32 + k));
            } else {
                lft[k] = from_lower_z(v[VX - R + k]);
                rgt[k] = from_upper_z(v[k]);
            }
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
    // (The last level skips this: ghost cells are never stored and the store
    // rounds.)
    template <bool FAST>
    static __device__ __forceinline__ void finish(const Ctx& c, int32_t y, TC (&out)[VX]) {
        const bool yg = ghost(y, c.ny);
#pragma unroll
        for (int e = 0; e < VX; ++e) {
            const bool g = yg || (!FAST && ghost(c.xl + e, c.nx));
            out[e] = g ? TC(0) : S::round(out[e]);
        }
    }

    template <bool FAST>
    static __device__ __forceinline__ void store_row(const Ctx& c, int32_t y, const TC (&out)[VX]) {
        const bool ok = static_cast<uint32_t>(y - c.ys) < static_cast<uint32_t>(c.ye - c.ys);
        TS* base = ok ? c.dst + static_cast<int64_t>(y) * c.nx + c.ofirst : c.dst;
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(base, 0, ok ? c.out_bytes : 0, kRsrcWord3);
        if constexpr (FAST) {
            bstorev(r, c.so, out);
        } else {
#pragma unroll
            for (int e = 0; e < VX; ++e) bstore1(r, c.so + e * static_cast<uint32_t>(sizeof(TS)), out[e]);
        }
    }

    template <int TB>
    struct State {
        TC q[TB][Q][VX];
        TC xq[Q];           // step-0 ring values of the queued rows
        TC pf[Q][VX];
        TC pfx[Q];
        int32_t yl;         // next row to load (wrapped when periodic)
        double fl;          // FLX: outflow through the y faces so far
        double xa[2];       // FLX: totals of the two candidate x-face columns
    };

    // Outflow (FLX: radius-1 star, zero rule, whole-vector rows).  The state
    // a step reads sends w_p * u(c) to c - off_p; a cell's leaving weight is
    // cy(y) + cx(x).  Canonical indices: y -1 is point 1, x -1 point 2, x +1
    // point 3, y +1 point 4; a point -1 along an axis sends to i + 1, a point
    // +1 to i - 1.  The y part is nonzero only on the first and last row (the
    // first and last y chunk), summed per cell in FP64 behind wave-uniform
    // branches; the x part only in column 0 (lane 0's first column: the
    // strip touching the face moves inward to start there) and column nx - 1
    // (lane 63's last), whose per-lane FP64 totals are weighted once at the
    // end.
    static_assert(!FLX || (R == 1 && CLS == kStar && !PER), "outflow variants: radius-1 star, zero rule");
    static __device__ __forceinline__ double leave_y(const Ctx& c, int32_t y) {
        return (y + 1 >= c.ny ? static_cast<double>(c.w[1]) : 0.0) + (y - 1 < 0 ? static_cast<double>(c.w[4]) : 0.0);
    }
    static __device__ __forceinline__ double leave_x(const Ctx& c, int32_t x) {
        return (x + 1 >= c.nx ? static_cast<double>(c.w[2]) : 0.0) + (x - 1 < 0 ? static_cast<double>(c.w[3]) : 0.0);
    }
    template <int TB, bool FAST>
    static __device__ __forceinline__ void flux_add(const Ctx& c, State<TB>& s, int32_t y, const TC (&v)[VX]) {
        if (static_cast<uint32_t>(y - c.ys) >= static_cast<uint32_t>(c.ye - c.ys)) return;
        if (c.fyb && (y < 1 || y >= c.ny - 1)) {
            const double cy = leave_y(c, y);
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                const bool own = static_cast<uint32_t>(c.xl + e - c.ofirst) < static_cast<uint32_t>(c.olast - c.ofirst);
                // opaque copy: keeps the conversion inside this rare branch
                TC u = v[e];
                __asm__ volatile("" : "+v"(u));
                s.fl = own ? fma(static_cast<double>(u), cy, s.fl) : s.fl;
            }
        }
        if (c.fx) {
            if constexpr (FAST) {
                s.xa[0] += static_cast<double>(v[0]);
                s.xa[1] += static_cast<double>(v[VX - 1]);
            } else {
                // element-wise rows (narrow or unaligned grids): any column
#pragma unroll
                for (int e = 0; e < VX; ++e) {
                    const int32_t x = c.xl + e;
                    const bool own = static_cast<uint32_t>(x - c.ofirst) < static_cast<uint32_t>(c.olast - c.ofirst);
                    s.fl = own ? fma(static_cast<double>(v[e]), leave_x(c, x), s.fl) : s.fl;
                }
            }
        }
    }
    template <int TB, bool FAST>
    static __device__ __forceinline__ void flux_store(const Ctx& c, const State<TB>& s) {
        double t = s.fl;
        if constexpr (FAST) {
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int32_t x = c.xl + (i == 0 ? 0 : VX - 1);
                const bool own = static_cast<uint32_t>(x - c.ofirst) < static_cast<uint32_t>(c.olast - c.ofirst);
                t = fma(s.xa[i], own ? leave_x(c, x) : 0.0, t);
            }
        }
        t = wave_sum(t);
        if (c.lane == 0) *c.fpart = t;
    }

    // Tessellated tiling along y (paper Sec. 4.1: triangles, then inverted
    // triangles from two halves of neighbouring triangles).  A chunk streams
    // only its own rows, so state s of row y is exact only at distance
    // >= R*s from a junction (a chunk boundary shared with another chunk);
    // the row's last exact state is L = min(T_b, d / R).  Rows with L = T_b
    // are stored as usual; for the others the two highest exact states (L and
    // L - 1: "top" and "pen") go to the junction's band block, where stage 2
    // (tess2d.hip) finishes them.  State s of row y is kept when its distance
    // d lies in [R*s, R*s + 2R): top when d < R*(s + 1), pen otherwise; a
    // state-0 row also keeps its ring values (the R columns beyond each end
    // of the strip), so that stage 2's first step is exact on the whole strip
    // as stage 1's is.  Band block of (junction, strip): top [BR][W], pen
    // [BR][W], ring [BR][64]; band row b of junction J is grid row
    // J - R*(T_b + 1) + b.
    template <int TB, int SL>
    static __device__ __forceinline__ void tess_capture(const Ctx& c, int32_t y, const TC (&v)[VX], TC xr) {
        constexpr int BR = tess_band_rows(R, TB);
        constexpr int H = R * (TB + 1);
        const int32_t dlo = y - c.clo, dhi = c.chi - y;
        TS* blk;
        int32_t b, d;
        if (static_cast<uint32_t>(dlo - R * SL) < static_cast<uint32_t>(2 * R)) {
            blk = c.blo;
            b = H + dlo;
            d = dlo;
        } else if (static_cast<uint32_t>(dhi - R * SL) < static_cast<uint32_t>(2 * R)) {
            blk = c.bhi;
            b = H - 1 - dhi;
            d = dhi;
        } else {
            return;
        }
        TS* row = blk + ((d < R * (SL + 1) ? 0 : BR) + b) * W;
        const __amdgpu_buffer_rsrc_t r =
            __builtin_amdgcn_make_buffer_rsrc(row, 0, static_cast<uint32_t>(W * sizeof(TS)), kRsrcWord3);
        bstorev(r, static_cast<uint32_t>(c.lane * VX * sizeof(TS)), v);
        if constexpr (SL == 0) {
            TS* ring = blk + 2 * BR * W + b * 64;
            const __amdgpu_buffer_rsrc_t rr =
                __builtin_amdgcn_make_buffer_rsrc(ring, 0, static_cast<uint32_t>(64 * sizeof(TS)), kRsrcWord3);
            bstore1(rr, static_cast<uint32_t>(c.lane * sizeof(TS)), xr);
        }
    }

    // level index of an unrolled loop to the template argument
    template <int TB, int SL = 1>
    static __device__ __forceinline__ void tess_capture_l(const Ctx& c, int sl, int32_t y, const TC (&v)[VX]) {
        if constexpr (SL < TB) {
            if (sl == SL) tess_capture<TB, SL>(c, y, v, TC(0));
            else tess_capture_l<TB, SL + 1>(c, sl, y, v);
        }
    }

    static __device__ __forceinline__ int32_t next_row(const Ctx& c, int32_t y) {
        if constexpr (PER) return y + 1 == c.ny ? 0 : y + 1;
        return y + 1;
    }

    // CAP: the iteration may capture band rows (TESS: only the first 2R*T_b
    // and the last 2R iterations of a chunk do)
    template <int TB, bool FAST, int J, bool CAP = TESS>
    static __device__ __forceinline__ void step(const Ctx& c, int32_t it, int32_t yfirst, State<TB>& s) {
        const int32_t yin = yfirst + it;
#pragma unroll
        for (int e = 0; e < VX; ++e) s.q[0][J][e] = s.pf[J][e];
        s.xq[J] = s.pfx[J];
        if constexpr (FLX) flux_add<TB, FAST>(c, s, yin, s.q[0][J]);  // the pass's input state
        if constexpr (TESS && CAP) tess_capture<TB, 0>(c, yin, s.q[0][J], s.xq[J]);
        // rows past the end of the stream are never consumed: load the last
        // streamed row again (a cache hit)
        load_row<FAST>(c, yin + Q <= c.ylast ? s.yl : c.ylast_w, s.pf[J], s.pfx[J]);
        s.yl = next_row(c, s.yl);
#pragma unroll
        for (int l = 0; l < TB; ++l) {
            TC out[VX];
            if (l == 0) compute<J, true>(c, s.q[0], s.xq, out);
            else compute<J, false>(c, s.q[l], s.xq, out);
            const int32_t yc = yin - (l + 1) * R;
            if (l + 1 == TB) {
                store_row<FAST>(c, yc, out);
            } else {
                finish<FAST>(c, yc, out);
                if constexpr (FLX) flux_add<TB, FAST>(c, s, yc, out);  // state after step l
                if constexpr (TESS && CAP) tess_capture_l<TB>(c, l + 1, yc, out);
#pragma unroll
                for (int e = 0; e < VX; ++e) s.q[l + 1][J][e] = out[e];
            }
        }
    }

    template <int TB, bool FAST, bool CAP, int... J>
    static __device__ __forceinline__ void group(const Ctx& c, int32_t base, int32_t yfirst, State<TB>& s,
                                                 std::integer_sequence<int, J...>) {
        (step<TB, FAST, J, CAP>(c, base + J, yfirst, s), ...);
    }
    template <int TB, bool FAST, int... J>
    static __device__ __forceinline__ void tail(const Ctx& c, int32_t base, int32_t nit, int32_t yfirst,
                                                State<TB>& s, std::integer_sequence<int, J...>) {
        ((base + J < nit ? step<TB, FAST, J>(c, base + J, yfirst, s) : void()), ...);
    }

    static __device__ __forceinline__ int32_t wrap_row(const Ctx& c, int32_t y) {
        return PER ? wrap_idx(y, c.ny) : y;
    }

    template <int TB, bool FAST>
    static __device__ __forceinline__ void body(Ctx& c) {
        // TESS: a junction side streams no halo rows (the triangle); a grid
        // edge under the zero rule streams the ghost rows as usual
        const int32_t yfirst = TESS ? (c.jlo ? c.cs : c.cs - R * TB) : c.ys - R * TB;
        const int32_t nit = TESS ? (c.jhi ? c.ce : c.ce + R * TB) - yfirst : (c.ye - c.ys) + 2 * R * TB;
        c.ylast = yfirst + nit - 1;
        c.ylast_w = wrap_row(c, c.ylast);
        State<TB> s;
#pragma unroll
        for (int l = 0; l < TB; ++l)
#pragma unroll
            for (int sl = 0; sl < Q; ++sl)
#pragma unroll
                for (int e = 0; e < VX; ++e) s.q[l][sl][e] = TC(0);
        s.yl = wrap_row(c, yfirst);
        s.fl = 0.0;
        s.xa[0] = s.xa[1] = 0.0;
#pragma unroll
        for (int sl = 0; sl < Q; ++sl) {
            s.xq[sl] = TC(0);
            load_row<FAST>(c, yfirst + sl <= c.ylast ? s.yl : c.ylast_w, s.pf[sl], s.pfx[sl]);
            s.yl = next_row(c, s.yl);
        }
        int32_t base = 0;
        if constexpr (TESS) {
            // the capture windows: state SL of a row at distance d in
            // [R*SL, R*SL + 2R) from a junction is made R*SL rows after the
            // row is loaded, so captures happen only in the first 2R*T_b
            // iterations (junction above) and the last 2R (junction below)
            const int32_t head = 2 * R * TB, tail0 = nit - 2 * R;
            for (; base + Q <= nit && base < head; base += Q)
                group<TB, FAST, true>(c, base, yfirst, s, std::make_integer_sequence<int, Q>{});
            for (; base + Q <= tail0; base += Q)
                group<TB, FAST, false>(c, base, yfirst, s, std::make_integer_sequence<int, Q>{});
            for (; base + Q <= nit; base += Q)
                group<TB, FAST, true>(c, base, yfirst, s, std::make_integer_sequence<int, Q>{});
        } else {
            for (; base + Q <= nit; base += Q)
                group<TB, FAST, false>(c, base, yfirst, s, std::make_integer_sequence<int, Q>{});
        }
        tail<TB, FAST>(c, base, nit, yfirst, s, std::make_integer_sequence<int, Q>{});
        if constexpr (FLX) flux_store<TB, FAST>(c, s);
    }

    // one specialised pipeline per fused depth
    template <bool FAST>
    static __device__ __forceinline__ void dispatch(Ctx& c, int tb) {
        if constexpr (TBMAX >= 8) if (tb == 8) return body<8, FAST>(c);
        if constexpr (TBMAX >= 7) if (tb == 7) return body<7, FAST>(c);
        if constexpr (TBMAX >= 6) if (tb == 6) return body<6, FAST>(c);
        if constexpr (TBMAX >= 5) if (tb == 5) return body<5, FAST>(c);
        if constexpr (TBMAX >= 4) if (tb == 4) return body<4, FAST>(c);
        if constexpr (TBMAX >= 3) if (tb == 3) return body<3, FAST>(c);
        if constexpr (TBMAX >= 2) if (tb == 2) return body<2, FAST>(c);
        body<1, FAST>(c);
    }

    // everything is inlined into the kernel: no device-function calls
    static __device__ __forceinline__ void run(const Stream2DArgs& a) {
        const int lane = threadIdx.x & 63;
        const int64_t wg = xcd_remap(blockIdx.x, gridDim.x);
        const int64_t item = __builtin_amdgcn_readfirstlane(static_cast<int>(wg * 4 + (threadIdx.x >> 6)));
        if (item >= a.items) return;
        const Stream2DGrid* gp = &a.one;
        int tb;
        bool odd = false;
        if (a.grids != nullptr) {
            int lo = 0, hi = a.ngrids - 1;
            while (lo < hi) {  // last grid whose tile_begin <= item
                const int mid = (lo + hi + 1) >> 1;
                if (a.grids[mid].tile_begin <= item) lo = mid; else hi = mid - 1;
            }
            gp = a.grids + lo;
            // this grid's depth at pass a.pass: `full` passes of depth tb,
            // then its tail passes; none left = nothing to do
            const int32_t full = uni(gp->full);
            const int32_t j = a.pass - full;
            tb = j < 0 ? uni(gp->tb) : (j == 0 ? uni(gp->tail[0]) : (j == 1 ? uni(gp->tail[1]) : (j == 2 ? uni(gp->tail[2]) : 0)));
            odd = (a.pass & 1) != 0;
            if (tb <= 0) {
                if constexpr (FLX) {
                    if (lane == 0) a.flux_part[item] = 0.0;
                }
                return;
            }
        } else {
            // the descriptor may live in global memory: pin every field to SGPRs
            tb = uni(gp->tb);
        }
        const int32_t tiles_x = uni(gp->tiles_x);
        const int32_t out_w = uni(gp->out_w);
        const int32_t hxa = uni(gp->hxa);
        const int32_t chunk_y = uni(gp->chunk_y);
        const bool vec_ok = uni(gp->vec_ok) != 0;
        Ctx c;
        // odd batch passes run from the work buffer back into the grid
        c.src = static_cast<const TS*>(odd ? uni(gp->dst) : uni(gp->src));
        c.dst = static_cast<TS*>(odd ? uni(const_cast<void*>(gp->src)) : uni(gp->dst));
        c.ny = static_cast<int32_t>(uni(gp->ny));
        c.nx = static_cast<int32_t>(uni(gp->nx));
        c.row_bytes = static_cast<uint32_t>(c.nx) * sizeof(TS);
        c.lane = lane;
        const int32_t local = static_cast<int32_t>(item - uni(gp->tile_begin));
        const int32_t cy = local / tiles_x, tx = local - cy * tiles_x;
        c.ofirst = tx * out_w;
        c.olast = c.ofirst + out_w < c.nx ? c.ofirst + out_w : c.nx;
        c.X0 = c.ofirst - hxa;
        const bool fast = vec_ok && (PER || c.nx >= W);
        if (!PER && fast) c.X0 = c.X0 < 0 ? 0 : (c.X0 + W > c.nx ? c.nx - W : c.X0);
        c.xl = c.X0 + lane * VX;
        // 32-bit offsets within a row: a ghost column becomes a huge unsigned
        // offset, past the end of the row's range
        c.lo = static_cast<uint32_t>(PER ? wrap_idx(c.xl, c.nx) : c.xl) * sizeof(TS);
#pragma unroll
        for (int e = 0; e < VX; ++e)
            c.eo[e] = static_cast<uint32_t>(PER ? wrap_idx(c.xl + e, c.nx) : c.xl + e) * sizeof(TS);
        {
            const bool right = lane >= 32;
            const int k = right ? lane - 32 : lane;
            const int32_t xr_x = right && k < R ? c.X0 + W + k : c.X0 - R + (k < R ? k : 0);
            c.xr_off = static_cast<uint32_t>(PER ? wrap_idx(xr_x, c.nx) : xr_x) * sizeof(TS);
        }
        c.so = static_cast<uint32_t>(c.xl - c.ofirst) * sizeof(TS);
        c.out_bytes = static_cast<uint32_t>(c.olast - c.ofirst) * sizeof(TS);
        c.ys = cy * chunk_y;
        c.ye = c.ys + chunk_y < c.ny ? c.ys + chunk_y : c.ny;
        if constexpr (TESS) {
            // chunks of chunk_y rows, the last one taking the remainder; a
            // junction between every two chunks (and, periodic, between the
            // last and the first); rows within R*tb of a junction are
            // finished by stage 2
            const int32_t chunks = uni(gp->chunks_y);
            c.cs = c.ys;
            c.ce = cy + 1 == chunks ? c.ny : c.ys + chunk_y;
            c.jlo = PER || cy > 0;
            c.jhi = PER || cy + 1 < chunks;
            constexpr int32_t kFar = -(1 << 29);
            c.clo = c.jlo ? c.cs : kFar;
            c.chi = c.jhi ? c.ce - 1 : kFar;
            // junction j sits above chunk j (periodic: junction 0 also below
            // the last chunk)
            const int64_t blk = static_cast<int64_t>(tess_band_rows(R, tb)) * (2 * W + 64);
            TS* const t0 = static_cast<TS*>(a.tess);
            c.blo = t0 + (static_cast<int64_t>(cy) * tiles_x + tx) * blk;
            c.bhi = t0 + (static_cast<int64_t>(cy + 1 == chunks ? 0 : cy + 1) * tiles_x + tx) * blk;
            c.ys = c.cs + (c.jlo ? R * tb : 0);
            c.ye = c.ce - (c.jhi ? R * tb : 0);
        }
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            c.w[p] = static_cast<TC>(uni(gp->w[p]));
            // TESS with many weights (the radius-2 boxes): the weights live
            // in VGPRs, leaving the scalar registers to the capture code
            if constexpr (TESS && NP * sizeof(TC) > 96) __asm__ volatile("" : "+v"(c.w[p]));
        }
        if constexpr (FLX) {
            c.fpart = a.flux_part + item;
            c.fx = c.ofirst < 1 || c.olast > c.nx - 1;
            c.fyb = c.ys < 1 || c.ye > c.ny - 1;
        }
        if (fast) dispatch<true>(c, tb);
        else dispatch<false>(c, tb);
    }
};

template <typename TS, int R, int CLS, int TBMAX, int VX, bool PER, bool FLX, bool TESS = false>
__global__ __launch_bounds__(256) void stream2d_kernel(const Stream2DArgs a) {
    Kern<TS, R, CLS, TBMAX, VX, PER, FLX, TESS>::run(a);
}

template <typename TS, int R, int CLS, int TBMAX, int VX, bool PER, bool FLX, bool TESS = false>
void launch(const Stream2DArgs& a, hipStream_t s) {
    const int64_t wgs = (a.items + 3) / 4;
    hipLaunchKernelGGL((stream2d_kernel<TS, R, CLS, TBMAX, VX, PER, FLX, TESS>), dim3(static_cast<unsigned>(wgs)),
                       dim3(256), 0, s, a);
}

template <typename TS, int R, int CLS, int TBMAX, int VX, bool PER, bool FLX, bool TESS = false>
int occ_of() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, stream2d_kernel<TS, R, CLS, TBMAX, VX, PER, FLX, TESS>, 256,
                                                     0) != hipSuccess)
        n = 0;
    return n;
}

template <typename TS> constexpr int32_t dtype_of();
template <> constexpr int32_t dtype_of<double>() { return kF64; }
template <> constexpr int32_t dtype_of<float>() { return kF32; }
template <> constexpr int32_t dtype_of<bf16s>() { return kBF16; }

#define S2D_ENTRY(TS, R, CLS, TBM, VX, PER, FLX)                                               \
    Entry2{Stream2DKey{dtype_of<TS>(), (PER) ? kPeriodic : kZero, CLS, R, TBM, VX, FLX, 0},    \
           &launch<TS, R, CLS, TBM, VX, PER, FLX>, &occ_of<TS, R, CLS, TBM, VX, PER, FLX>}
// stage 1 of the tessellated tiling (stage 2: tess2d.hip)
#define S2D_TESS_ENTRY(TS, R, CLS, TBM, VX, PER)                                                \
    Entry2{Stream2DKey{dtype_of<TS>(), (PER) ? kPeriodic : kZero, CLS, R, TBM, VX, 0, 1},       \
           &launch<TS, R, CLS, TBM, VX, PER, false, true>, &occ_of<TS, R, CLS, TBM, VX, PER, false, true>}
#define S2D_TESS(TS, R, CLS, TBM, VX) S2D_TESS_ENTRY(TS, R, CLS, TBM, VX, false), S2D_TESS_ENTRY(TS, R, CLS, TBM, VX, true)
#define S2D_BC(TS, R, CLS, TBM, VX) \
    S2D_ENTRY(TS, R, CLS, TBM, VX, false, false), S2D_ENTRY(TS, R, CLS, TBM, VX, true, false)
// outflow-summing variant (radius-1 star, zero rule, single grid)
#define S2D_FLUX(TS, TBM, VX) S2D_ENTRY(TS, 1, kStar, TBM, VX, false, true)

}  // namespace s2d
}  // namespace st
