// stream3d_impl.h -- 3D star stencils (radius R) with T_b steps fused per pass.
//
// 2.5-D blocking: an xy tile is held on chip while the work-group streams
// along z (paper Sec. 4.1 builds space-time tiles, tetrahedra in 3D; Sec. 4.2
// stages tiles on chip so global accesses stay coalesced).  On gfx950 the
// on-chip tile lives in VGPRs:
//   * lane L of wave w holds columns X0 + L*VX .. +VX-1 of rows
//     Y0 + w*K .. Y0 + w*K + K-1 (one 16-byte access per row);
//   * pipeline level l keeps the last 2R+1 planes of step l (its z queue);
//   * x neighbours: own registers, or lane +-1 through DPP.  The R columns
//     just outside the tile (step 0 only) are fetched for all K rows by one
//     load instruction (lanes 0.. and 32.. each fetch one value) and enter the
//     DPP "old" operand of lanes 0 and 63 through readlane;
//   * y neighbours of step 0: own rows, plus R rows above and R rows below
//     the wave's rows loaded directly (they are other waves' rows, so the
//     loads hit in cache) -- or, in the YL variants, the edge rows of the
//     neighbouring waves through LDS, the tile's own 2R halo rows being
//     loaded once per tile (split over the waves) instead of once per wave;
//     of steps >= 1 (T_b > 1): the edge rows of the neighbouring waves,
//     exchanged through LDS once per level and plane;
//   * z neighbours: queue slots.
// Loads run P planes ahead of use (P = 3 when 2R+1 is a multiple of 3) and
// are unconditional buffer loads: each row is read through a descriptor whose
// byte range is that row (the whole plane for the x-ring values), and a row or
// plane outside the grid gets an empty range, so under the zero rule the
// hardware returns 0 for every ghost cell -- no masks, no clamped indices, and
// no branch between a load and its use to drain the prefetch.  Lanes address
// their columns with a 32-bit offset fixed for the whole run (no 64-bit
// per-lane pointers), which needs planes below 2 GiB.
//
// Tiles.  Step l is exact on the register tile shrunk by (l-1)*R per side
// (hxa, hya >= R*(tb-1) columns/rows of halo are stored by the neighbour
// tile).  Under the zero rule a tile that would cross the grid edge is moved
// inward to touch it instead: the ghost layer outside the grid is 0 at every
// step (lanes 0/63 get 0 from DPP, the LDS ring rows hold 0), so the tile
// stays exact up to the edge.  Under the periodic rule tiles keep their
// place and every index wraps.  A z chunk [zs, ze) streams planes
// zs - R*tb .. ze - 1 + R*tb.
//
// FAST = whole-vector row access (nx % VX == 0, 16-byte aligned base, and
// under the zero rule nx >= 64*VX, ny >= NW*K); otherwise every element is
// loaded and stored on its own, with the same arithmetic.
#pragma once

#include <utility>

#include "dev_common.h"
#include "registry.h"

namespace st {

namespace s3d {

template <typename TS, int R, int TBMAX, int VX, int K, int NW, bool PER, bool FAST, bool LATE, bool YL, bool FLX>
struct Kern {
    using S = Storage<TS>;
    using TC = typename S::TC;
    static_assert(VX >= R, "a lane must hold at least R columns");
    static_assert(K * R <= 32, "the x ring of a wave must fit in half a wave");
    static constexpr int Q = 2 * R + 1;
    // Prefetch: P planes ahead into their own registers, or (LATE) one plane
    // ahead straight into the step-0 queue slot that step 0 has just
    // released, issued after step 0 so the deeper steps hide its latency.
    static constexpr int P = LATE ? 1 : ((Q % 3 == 0) ? 3 : Q);
    static constexpr int PR = (R == 1 && !LATE) ? P : 1;  // ring prefetch depth
    static constexpr int W = 64 * VX;
    static constexpr int H = NW * K;
    static constexpr int NP = 6 * R + 1;
    static constexpr int SLOTS = H + 2 * R;              // LDS rows -R .. H+R-1
    static constexpr int BUF_ELEMS = SLOTS * W;
    // YL: halo rows of the tile each wave loads (slots beyond 2R repeat the last)
    static constexpr int HR = YL ? (2 * R + NW - 1) / NW : 0;
    static constexpr int RROWS = YL ? HR : 2 * R;         // ring rows per prefetch slot
    static constexpr bool XCH = YL || TBMAX > 1;          // any LDS exchange
    static constexpr int LDS_BYTES = XCH ? 2 * BUF_ELEMS * static_cast<int>(sizeof(TC)) : 0;

    struct Ctx {
        const TS* src;
        int32_t nz, ny, nx;          // every index fits 32 bits: planes are below 2^31 bytes
        int64_t plane_elems;
        int32_t X0, Y0;
        int32_t xl;            // first column of this lane
        int32_t yw;            // first row of this wave
        int32_t zs, ze, zlast; // output planes [zs, ze); last streamed plane
        int32_t ox0, ox1, oy0, oy1;
        int32_t xr_x, xr_y;    // the x-ring element this lane fetches
        int32_t hy[HR > 0 ? HR : 1];   // YL: grid rows of this wave's halo rows
        int hslot[HR > 0 ? HR : 1];    // YL: their LDS slots
        int32_t yk[K];                 // rows this wave loads (wrapped when periodic)
        int32_t yr[2 * R];             // its ring rows above and below (not YL)
        int32_t yh[HR > 0 ? HR : 1];   // YL halo rows as loaded
        uint32_t row_bytes, plane_bytes;
        uint32_t lo;                   // byte offset of this lane's first column in a row
        uint32_t eo[VX];               // element offsets (element-wise access)
        uint32_t xr_off;               // byte offset of the x-ring element in its plane
        bool xr_xg;                    // that element is an x ghost (zero rule)
        TS* dstg;                      // output grid (buffer stores)
        uint32_t so;                   // byte offset of this lane's first column from ox0
        uint32_t out_bytes;            // bytes of one output row of the tile
        int lane, wave;
        TC w[NP];
        double* fpart;                 // FLX: this wave's partial outflow slot
        bool fx;                       // FLX: the output tile is within R of an x face
        bool fy;                       // FLX: this wave's owned rows reach within R of a y face
        bool fzy;                      // FLX: fy, or the z chunk reaches within R of a z face
        TC rw[K];                      // FLX: 1 for the wave's owned rows, 0 for the others
    };

    static __device__ __forceinline__ bool ghost(int32_t i, int32_t n) {
        return !PER && static_cast<uint32_t>(i) >= static_cast<uint32_t>(n);  // i < 0 or i >= n
    }
    static __device__ __forceinline__ int32_t wz(int32_t z, int32_t n) { return PER ? wrap_idx(z, n) : z; }

    // Descriptors: one row of plane zz (or the whole plane); empty outside the
    // grid.  Periodic indices arrive wrapped.
    static constexpr int32_t kRsrcWord3 = 0x00020000;  // gfx9: raw 32-bit data
    static constexpr int32_t kNT = 2;                  // store cache policy: non-temporal
    static __device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const Ctx& c, int32_t zz, int32_t y) {
        const bool out = ghost(zz, c.nz) || ghost(y, c.ny);
        const TS* base = out ? c.src : c.src + static_cast<int64_t>(zz) * c.plane_elems + y * c.nx;
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<TS*>(base), 0, out ? 0 : c.row_bytes, kRsrcWord3);
    }
    static __device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const Ctx& c, int32_t zz) {
        const bool out = ghost(zz, c.nz);
        const TS* base = out ? c.src : c.src + static_cast<int64_t>(zz) * c.plane_elems;
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<TS*>(base), 0, out ? 0 : c.plane_bytes, kRsrcWord3);
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

    static __device__ __forceinline__ void load_row(const Ctx& c, int32_t zz, int32_t y, TC (&v)[VX]) {
        const __amdgpu_buffer_rsrc_t r = row_rsrc(c, zz, y);
        if constexpr (FAST) {
            bloadv(r, c.lo, v);
        } else {
#pragma unroll
            for (int e = 0; e < VX; ++e) v[e] = bload1(r, c.eo[e]);
        }
    }

    // Loads of one pipeline slot: the wave's K rows of plane zm, and the ring
    // (2R rows, or the wave's share of the tile halo with YL, and one x-ring
    // value per lane) of plane zr.  Planes past the end of the stream repeat
    // its last plane (cache hits).
    static __device__ __forceinline__ void load_main(const Ctx& c, int32_t zm, TC (&v)[K][VX]) {
        const int32_t zz = wz(zm < c.zlast ? zm : c.zlast, c.nz);
#pragma unroll
        for (int k = 0; k < K; ++k) load_row(c, zz, c.yk[k], v[k]);
    }
    static __device__ __forceinline__ void load_ring(const Ctx& c, int32_t zr, TC (&r)[RROWS][VX], TC& xv) {
        const int32_t zz = wz(zr < c.zlast ? zr : c.zlast, c.nz);
        if constexpr (YL) {
#pragma unroll
            for (int j = 0; j < HR; ++j) load_row(c, zz, c.yh[j], r[j]);
        } else {
#pragma unroll
            for (int j = 0; j < 2 * R; ++j) load_row(c, zz, c.yr[j], r[j]);
        }
        xv = bload1(plane_rsrc(c, zz), c.xr_off);
    }

    // Consuming a slot: the loads already hold 0 on the ghost layer, except
    // the x-ring value of a lane whose column lies outside the grid (it would
    // otherwise read the neighbouring row).
    static __device__ __forceinline__ void take_main(const Ctx&, int32_t, const TC (&v)[K][VX], TC (&q)[K][VX]) {
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int e = 0; e < VX; ++e) q[k][e] = v[k][e];
    }
    static __device__ __forceinline__ void take_ring(const Ctx& c, int32_t, const TC (&r)[RROWS][VX], TC xv,
                                                     TC (&above)[R][VX], TC (&below)[R][VX], TC& xg) {
        static_assert(!YL, "the YL variants take their halo rows with take_halo");
#pragma unroll
        for (int j = 0; j < R; ++j)
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                above[j][e] = r[j][e];
                below[j][e] = r[R + j][e];
            }
        xg = c.xr_xg ? TC(0) : xv;
    }
    static __device__ __forceinline__ void take_halo(const Ctx& c, int32_t, const TC (&r)[RROWS][VX], TC xv,
                                                     TC (&h)[RROWS][VX], TC& xg) {
#pragma unroll
        for (int j = 0; j < RROWS; ++j)
#pragma unroll
            for (int e = 0; e < VX; ++e) h[j][e] = r[j][e];
        xg = c.xr_xg ? TC(0) : xv;
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

    static __device__ __forceinline__ TC xval(const TC (&v)[VX], const TC (&lft)[R],
                                              const TC (&rgt)[R], int idx) {
        return idx < 0 ? lft[R + idx] : (idx >= VX ? rgt[idx - VX] : v[idx]);
    }

    // Step l+1 on the centre plane of queue q (slot (J-R) mod Q).  Canonical
    // point order for a 3D star: centre; z -R..-1; y -R..-1; x -R..-1;
    // x +1..+R; y +1..+R; z +1..+R.
    template <int J, bool LEVEL0>
    static __device__ __forceinline__ void compute(const Ctx& c, const TC (&q)[Q][K][VX], TC xg,
                                                   const TC (&above)[R][VX], const TC (&below)[R][VX],
                                                   TC (&out)[K][VX]) {
        constexpr int CEN = (J - R + Q) % Q;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            TC lft[R], rgt[R];
#pragma unroll
            for (int j = 0; j < R; ++j) {
                if constexpr (LEVEL0) {
                    lft[j] = from_lower(q[CEN][k][VX - R + j], lane_value(xg, k * R + j));
                    rgt[j] = from_upper(q[CEN][k][j], lane_value(xg, 32 + k * R + j));
                } else {
                    lft[j] = from_lower_z(q[CEN][k][VX - R + j]);
                    rgt[j] = from_upper_z(q[CEN][k][j]);
                }
            }
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                TC acc = c.w[0] * q[CEN][k][e];
                int p = 1;
#pragma unroll
                for (int dz = -R; dz <= -1; ++dz, ++p)
                    acc = fma_c(c.w[p], q[(J - R + dz + 2 * Q) % Q][k][e], acc);
#pragma unroll
                for (int dy = -R; dy <= -1; ++dy, ++p) {
                    const int kk = k + dy;
                    const TC v = kk >= 0 ? q[CEN][kk >= 0 ? kk : 0][e] : above[R + (kk < 0 ? kk : -R)][e];
                    acc = fma_c(c.w[p], v, acc);
                }
#pragma unroll
                for (int dx = -R; dx <= -1; ++dx, ++p)
                    acc = fma_c(c.w[p], xval(q[CEN][k], lft, rgt, e + dx), acc);
#pragma unroll
                for (int dx = 1; dx <= R; ++dx, ++p)
                    acc = fma_c(c.w[p], xval(q[CEN][k], lft, rgt, e + dx), acc);
#pragma unroll
                for (int dy = 1; dy <= R; ++dy, ++p) {
                    const int kk = k + dy;
                    const TC v = kk < K ? q[CEN][kk < K ? kk : K - 1][e] : below[kk >= K ? kk - K : 0][e];
                    acc = fma_c(c.w[p], v, acc);
                }
#pragma unroll
                for (int dz = 1; dz <= R; ++dz, ++p)
                    acc = fma_c(c.w[p], q[(J - R + dz + 2 * Q) % Q][k][e], acc);
                out[k][e] = acc;
            }
        }
    }

    // Zero rule: ghost cells stay 0; bfloat16 storage rounds every step.  (The
    // last level skips this: its ghost cells are never stored and the store
    // rounds.)
    static __device__ __forceinline__ void finish(const Ctx& c, int32_t z, TC (&out)[K][VX]) {
        const bool zg = ghost(z, c.nz);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const bool rg = zg || (!FAST && ghost(c.yw + k, c.ny));
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                const bool g = rg || (!FAST && ghost(c.xl + e, c.nx));
                out[k][e] = g ? TC(0) : S::round(out[k][e]);
            }
        }
    }

    // Buffer stores through a descriptor per row whose range is the tile's
    // output columns of that row, or empty when the row or plane is not an
    // output: the hardware drops the rest, so every iteration issues the same
    // stores with no branch (and the wait counts stay exact).
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
    static __device__ __forceinline__ void store_plane(const Ctx& c, int32_t z, const TC (&out)[K][VX]) {
        const bool zok = static_cast<uint32_t>(z - c.zs) < static_cast<uint32_t>(c.ze - c.zs);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int32_t y = c.yw + k;
            const bool ok = zok && static_cast<uint32_t>(y - c.oy0) < static_cast<uint32_t>(c.oy1 - c.oy0);
            TS* base = ok ? c.dstg + static_cast<int64_t>(z) * c.plane_elems + y * c.nx + c.ox0 : c.dstg;
            const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(base, 0, ok ? c.out_bytes : 0, kRsrcWord3);
            if constexpr (FAST) {
                bstorev(r, c.so, out[k]);
            } else {
#pragma unroll
                for (int e = 0; e < VX; ++e) bstore1(r, c.so + e * static_cast<uint32_t>(sizeof(TS)), out[k][e]);
            }
        }
    }

    // Outflow (FLX, zero rule): the state a step reads sends w_p * u(c) to
    // c - off_p; for a star only the points along one axis can cross that
    // axis's faces.  Points -d (canonical index lo + R - d) send to i + d,
    // points +d (index hi + d - 1) to i - d.
    static __device__ __forceinline__ double leave_w(const Ctx& c, int32_t i, int32_t n, int lo, int hi) {
        double s = 0.0;
#pragma unroll
        for (int d = 1; d <= R; ++d) {
            if (i + d >= n) s += static_cast<double>(c.w[lo + R - d]);
            if (i - d < 0) s += static_cast<double>(c.w[hi + d - 1]);
        }
        return s;
    }
    template <int TB>
    struct State {
        TC q[TB][Q][K][VX];
        TC pf[LATE ? 1 : P][K][VX];  // unused when LATE
        TC rpf[PR][RROWS][VX];
        TC xpf[PR];
        double fl;                   // FLX: outflow of this wave's owned cells so far (z and y parts)
        double xa[(FAST && R == 1) ? 2 : VX];  // FLX: owned-row sums of the candidate face columns
    };

    // Adds the outflow of the wave's owned cells of plane z of one state:
    // sum over cells of u * (cz + cy + cx).
    //   * z and y parts (nonzero on the band planes, and on the band rows of
    //     the one or two waves per edge tile that own them): FP64 per cell,
    //     behind wave-uniform branches;
    //   * x part (every plane of the x-edge tiles): per candidate column, the
    //     sum over the owned rows of the plane (K values, in the compute
    //     precision) is added to an FP64 per-lane column total; the totals
    //     are weighted once, when the wave stores its partial sum.  With
    //     radius 1 in the whole-vector layout a face column is the first
    //     column of lane 0 or the last of lane 63 (edge tiles move inward to
    //     touch the faces, and only they own a face column), so only those
    //     two columns are candidates.
    static constexpr bool XEDGE2 = FAST && R == 1;
    static constexpr int NXB = XEDGE2 ? 2 : VX;
    static __device__ __forceinline__ int xcol(int i) { return XEDGE2 ? (i == 0 ? 0 : VX - 1) : i; }
    template <int TB>
    static __device__ __forceinline__ void flux_add(const Ctx& c, State<TB>& s, int32_t z, const TC (&v)[K][VX]) {
        if (static_cast<uint32_t>(z - c.zs) >= static_cast<uint32_t>(c.ze - c.zs)) return;
        if (c.fzy) {
            const bool zb = z < R || z >= c.nz - R;
            if (zb || c.fy) {
                const double cz = zb ? leave_w(c, z, c.nz, 1, 1 + 5 * R) : 0.0;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const int32_t y = c.yw + k;
                    if (static_cast<uint32_t>(y - c.oy0) >= static_cast<uint32_t>(c.oy1 - c.oy0)) continue;
                    const bool yb = y < R || y >= c.ny - R;
                    if (!zb && !yb) continue;
                    const double czy = yb ? cz + leave_w(c, y, c.ny, 1 + R, 1 + 4 * R) : cz;
#pragma unroll
                    for (int e = 0; e < VX; ++e) {
                        const bool own =
                            static_cast<uint32_t>(c.xl + e - c.ox0) < static_cast<uint32_t>(c.ox1 - c.ox0);
                        // opaque copy: keeps the conversion inside this rare
                        // branch (otherwise it is hoisted into every plane)
                        TC u = v[k][e];
                        __asm__ volatile("" : "+v"(u));
                        s.fl = own ? fma(static_cast<double>(u), czy, s.fl) : s.fl;
                    }
                }
            }
        }
        if (c.fx) {
#pragma unroll
            for (int i = 0; i < NXB; ++i) {
                TC col = c.rw[0] * v[0][xcol(i)];
#pragma unroll
                for (int k = 1; k < K; ++k) col = fma_c(c.rw[k], v[k][xcol(i)], col);
                s.xa[i] += static_cast<double>(col);
            }
        }
    }
    template <int TB>
    static __device__ __forceinline__ void flux_store(const Ctx& c, const State<TB>& s) {
        double t = s.fl;
#pragma unroll
        for (int i = 0; i < NXB; ++i) {
            const int32_t x = c.xl + xcol(i);
            const bool own = static_cast<uint32_t>(x - c.ox0) < static_cast<uint32_t>(c.ox1 - c.ox0);
            t = fma(s.xa[i], own ? leave_w(c, x, c.nx, 1 + 2 * R, 1 + 3 * R) : 0.0, t);
        }
        flux_store_sum(c, t);
    }
    static __device__ __forceinline__ void flux_store_sum(const Ctx& c, double fl) {
        const double t = wave_sum(fl);
        if (c.lane == 0) *c.fpart = t;
    }


    template <int TB, int J>
    static __device__ __forceinline__ void step(const Ctx& c, int32_t it, int32_t zfirst, State<TB>& s, TC* lds) {
        constexpr int SM = J % P, SR = J % PR;
        const int32_t zin = zfirst + it;
        // consume this iteration's slots, then refill them P (PR) planes ahead
        TC above0[R][VX], below0[R][VX], xg;
        TC halo[RROWS][VX];
        if constexpr (LATE) {
            take_main(c, zin, s.q[0][J], s.q[0][J]);
            if constexpr (YL) take_halo(c, zin - R, s.rpf[0], s.xpf[0], halo, xg);
            else take_ring(c, zin - R, s.rpf[0], s.xpf[0], above0, below0, xg);
        } else {
            take_main(c, zin, s.pf[SM], s.q[0][J]);
            if constexpr (YL) take_halo(c, zin - R, s.rpf[SR], s.xpf[SR], halo, xg);
            else take_ring(c, zin - R, s.rpf[SR], s.xpf[SR], above0, below0, xg);
            load_main(c, zin + P, s.pf[SM]);
            load_ring(c, zin + PR - R, s.rpf[SR], s.xpf[SR]);
        }
        if constexpr (FLX) flux_add(c, s, zin, s.q[0][J]);  // the pass's input state

        constexpr int CEN = (J - R + Q) % Q;
#pragma unroll
        for (int l = 0; l < TB; ++l) {
            {
                TC out[K][VX];
                if (l == 0 && !YL) {
                    compute<J, true>(c, s.q[0], xg, above0, below0, out);
                } else {
                    // exchange the edge rows of this level's centre plane; with
                    // YL every level's exchange also fills the 2R halo slots
                    // (step 0: the loaded halo rows, later steps: 0)
                    const int32_t seq = YL ? it * TB + l : it * (TB - 1) + (l - 1);
                    TC* buf = lds + (seq & 1) * BUF_ELEMS;
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        if (k < R || k >= K - R) {
                            TC* p = buf + (c.wave * K + k + R) * W + c.lane * VX;
#pragma unroll
                            for (int e = 0; e < VX; ++e) p[e] = s.q[l][CEN][k][e];
                        }
                    }
                    if constexpr (YL) {
#pragma unroll
                        for (int j = 0; j < HR; ++j) {
                            TC* p = buf + c.hslot[j] * W + c.lane * VX;
#pragma unroll
                            for (int e = 0; e < VX; ++e) p[e] = l == 0 ? halo[j][e] : TC(0);
                        }
                    }
                    __syncthreads();
                    TC above[R][VX], below[R][VX];
#pragma unroll
                    for (int j = 0; j < R; ++j) {
                        const TC* pa = buf + (c.wave * K + j) * W + c.lane * VX;
                        const TC* pb = buf + (c.wave * K + K + R + j) * W + c.lane * VX;
#pragma unroll
                        for (int e = 0; e < VX; ++e) {
                            above[j][e] = pa[e];
                            below[j][e] = pb[e];
                        }
                    }
                    if (l == 0) compute<J, true>(c, s.q[0], xg, above, below, out);
                    else compute<J, false>(c, s.q[l], TC(0), above, below, out);
                }
                if constexpr (LATE) {
                    if (l == 0) {
                        // step 0 no longer needs its oldest plane: load the next one there
                        load_main(c, zin + 1, s.q[0][(J + 1) % Q]);
                        load_ring(c, zin + 1 - R, s.rpf[0], s.xpf[0]);
                    }
                }
                const int32_t zc = zin - (l + 1) * R;
                if (l + 1 == TB) {
                    store_plane(c, zc, out);
                } else {
                    finish(c, zc, out);
                    if constexpr (FLX) flux_add(c, s, zc, out);  // state after step l
#pragma unroll
                    for (int k = 0; k < K; ++k)
#pragma unroll
                        for (int e = 0; e < VX; ++e) s.q[l + 1][J][k][e] = out[k][e];
                }
            }
        }
    }

    template <int TB, int... J>
    static __device__ __forceinline__ void group(const Ctx& c, int32_t base, int32_t zfirst, State<TB>& s, TC* lds,
                                                 std::integer_sequence<int, J...>) {
        (step<TB, J>(c, base + J, zfirst, s, lds), ...);
    }
    template <int TB, int... J>
    static __device__ __forceinline__ void tail(const Ctx& c, int32_t base, int32_t nit, int32_t zfirst,
                                                State<TB>& s, TC* lds, std::integer_sequence<int, J...>) {
        ((base + J < nit ? step<TB, J>(c, base + J, zfirst, s, lds) : void()), ...);
    }
    static __device__ __forceinline__ void run(const Stream3DArgs& a, TC* lds) {
        Ctx c;
        c.lane = threadIdx.x & 63;
        c.wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
        // work items < 2^31 (checked by the planner): 32-bit, once per work-group
        const uint32_t tiles = static_cast<uint32_t>(a.tiles_x) * a.tiles_y * a.chunks_z;
        const uint32_t item = static_cast<uint32_t>(xcd_remap(blockIdx.x, gridDim.x));
        if constexpr (FLX) c.fpart = a.flux_part + static_cast<int64_t>(blockIdx.x) * NW + c.wave;
        if (item >= tiles) {
            if constexpr (FLX) flux_store_sum(c, 0.0);
            return;
        }
        const uint32_t txy = item / static_cast<uint32_t>(a.tiles_x);
        const int32_t tx = static_cast<int32_t>(item - txy * a.tiles_x);
        const int32_t ty = static_cast<int32_t>(txy % static_cast<uint32_t>(a.tiles_y));
        const int32_t cz = static_cast<int32_t>(txy / static_cast<uint32_t>(a.tiles_y));
        c.src = static_cast<const TS*>(a.src);
        c.nz = static_cast<int32_t>(a.nz);
        c.ny = static_cast<int32_t>(a.ny);
        c.nx = static_cast<int32_t>(a.nx);
        c.plane_elems = a.ny * a.nx;
        c.ox0 = tx * a.out_w;
        c.oy0 = ty * a.out_h;
        c.ox1 = c.ox0 + a.out_w < c.nx ? c.ox0 + a.out_w : c.nx;
        c.oy1 = c.oy0 + a.out_h < c.ny ? c.oy0 + a.out_h : c.ny;
        c.X0 = c.ox0 - a.hxa;
        c.Y0 = c.oy0 - a.hya;
        if (!PER && FAST) {  // move edge tiles inward (exact: the ghost layer is 0)
            c.X0 = c.X0 < 0 ? 0 : (c.X0 + W > c.nx ? c.nx - W : c.X0);
            c.Y0 = c.Y0 < 0 ? 0 : (c.Y0 + H > c.ny ? c.ny - H : c.Y0);
        }
        c.xl = c.X0 + c.lane * VX;
        c.yw = c.Y0 + c.wave * K;
        {
            const bool right = c.lane >= 32;
            const int slot = right ? c.lane - 32 : c.lane;
            const int kr = slot < K * R ? slot / R : 0;
            const int jr = slot < K * R ? slot % R : 0;
            c.xr_y = c.yw + kr;
            c.xr_x = right && slot < K * R ? c.X0 + W + jr : c.X0 - R + jr;
        }
        if constexpr (YL) {
#pragma unroll
            for (int j = 0; j < HR; ++j) {
                const int h = c.wave * HR + j < 2 * R ? c.wave * HR + j : 2 * R - 1;
                c.hslot[j] = h < R ? h : H + h;
                c.hy[j] = c.Y0 + (c.hslot[j] - R);
                c.yh[j] = PER ? wrap_idx(c.hy[j], c.ny) : c.hy[j];
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) c.yk[k] = PER ? wrap_idx(c.yw + k, c.ny) : c.yw + k;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            c.yr[j] = PER ? wrap_idx(c.yw - R + j, c.ny) : c.yw - R + j;
            c.yr[R + j] = PER ? wrap_idx(c.yw + K + j, c.ny) : c.yw + K + j;
        }
        c.row_bytes = static_cast<uint32_t>(c.nx) * sizeof(TS);
        c.plane_bytes = static_cast<uint32_t>(c.plane_elems) * sizeof(TS);
        // 32-bit offsets: a ghost column or row becomes a huge unsigned offset,
        // past the end of the descriptor's range
        c.lo = static_cast<uint32_t>(PER ? wrap_idx(c.xl, c.nx) : c.xl) * sizeof(TS);
#pragma unroll
        for (int e = 0; e < VX; ++e)
            c.eo[e] = static_cast<uint32_t>(PER ? wrap_idx(c.xl + e, c.nx) : c.xl + e) * sizeof(TS);
        {
            const int32_t ry = PER ? wrap_idx(c.xr_y, c.ny) : c.xr_y;
            const int32_t rx = PER ? wrap_idx(c.xr_x, c.nx) : c.xr_x;
            c.xr_off = static_cast<uint32_t>(ry * c.nx + rx) * sizeof(TS);
            c.xr_xg = ghost(c.xr_x, c.nx);
        }
        c.dstg = static_cast<TS*>(a.dst);
        c.so = static_cast<uint32_t>(c.xl - c.ox0) * sizeof(TS);
        c.out_bytes = static_cast<uint32_t>(c.ox1 - c.ox0) * sizeof(TS);
        c.zs = cz * a.chunk_z;
        c.ze = c.zs + a.chunk_z < c.nz ? c.zs + a.chunk_z : c.nz;
#pragma unroll
        for (int p = 0; p < NP; ++p) c.w[p] = static_cast<TC>(a.w[p]);
        if constexpr (FLX) {
            c.fx = c.ox0 < R || c.ox1 > c.nx - R;
            c.fy = false;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int32_t y = c.yw + k;
                const bool own = static_cast<uint32_t>(y - c.oy0) < static_cast<uint32_t>(c.oy1 - c.oy0);
                c.fy = c.fy || (own && (y < R || y >= c.ny - R));
                c.rw[k] = own ? TC(1) : TC(0);
            }
            c.fzy = c.fy || c.zs < R || c.ze > c.nz - R;
        }
        // one specialised pipeline per fused depth: no run-time level tests
        // inside the loop
        const int tb = a.tb;
        if constexpr (TBMAX >= 4) if (tb == 4) return run_tb<4>(c, lds);
        if constexpr (TBMAX >= 3) if (tb == 3) return run_tb<3>(c, lds);
        if constexpr (TBMAX >= 2) if (tb == 2) return run_tb<2>(c, lds);
        run_tb<1>(c, lds);
    }

    template <int TB>
    static __device__ __forceinline__ void run_tb(Ctx& c, TC* lds) {
        const int32_t zfirst = c.zs - R * TB;
        const int32_t nit = (c.ze - c.zs) + 2 * R * TB;
        c.zlast = zfirst + nit - 1;

        if constexpr (TB > 1 && !YL) {
            // ring rows of every LDS buffer stay 0 (ghost / unused halo)
            for (int i = threadIdx.x; i < 2 * R * W; i += blockDim.x) {
                const int row = i / W, col = i % W;
                const int slot = row < R ? row : H + row;
                lds[slot * W + col] = TC(0);
                lds[BUF_ELEMS + slot * W + col] = TC(0);
            }
            __syncthreads();
        }

        State<TB> s;
        s.fl = 0.0;
#pragma unroll
        for (int i = 0; i < NXB; ++i) s.xa[i] = 0.0;
#pragma unroll
        for (int l = 0; l < TB; ++l)
#pragma unroll
            for (int sl = 0; sl < Q; ++sl)
#pragma unroll
                for (int k = 0; k < K; ++k)
#pragma unroll
                    for (int e = 0; e < VX; ++e) s.q[l][sl][k][e] = TC(0);
        if constexpr (LATE) {
            load_main(c, zfirst, s.q[0][0]);
            load_ring(c, zfirst - R, s.rpf[0], s.xpf[0]);
        } else {
#pragma unroll
            for (int sp = 0; sp < P; ++sp) load_main(c, zfirst + sp, s.pf[sp]);
#pragma unroll
            for (int sp = 0; sp < PR; ++sp) load_ring(c, zfirst + sp - R, s.rpf[sp], s.xpf[sp]);
        }

        int32_t base = 0;
        for (; base + Q <= nit; base += Q) group<TB>(c, base, zfirst, s, lds, std::make_integer_sequence<int, Q>{});
        tail<TB>(c, base, nit, zfirst, s, lds, std::make_integer_sequence<int, Q>{});
        if constexpr (FLX) flux_store(c, s);
    }
};

template <typename TS, int R, int TBMAX, int VX, int K, int NW, bool PER, bool FAST, bool LATE, bool YL, bool FLX>
__global__ __launch_bounds__(64 * NW) void stream3d_kernel(const Stream3DArgs a) {
    using KK = Kern<TS, R, TBMAX, VX, K, NW, PER, FAST, LATE, YL, FLX>;
    extern __shared__ __align__(16) unsigned char smem[];
    KK::run(a, reinterpret_cast<typename KK::TC*>(smem));
}

template <typename TS, int R, int TBMAX, int VX, int K, int NW, bool PER, bool FAST, bool LATE, bool YL, bool FLX>
void launch(const Stream3DArgs& a, hipStream_t s) {
    using KK = Kern<TS, R, TBMAX, VX, K, NW, PER, FAST, LATE, YL, FLX>;
    const int64_t tiles = static_cast<int64_t>(a.tiles_x) * a.tiles_y * a.chunks_z;
    hipLaunchKernelGGL((stream3d_kernel<TS, R, TBMAX, VX, K, NW, PER, FAST, LATE, YL, FLX>),
                       dim3(static_cast<unsigned>(tiles)), dim3(64 * NW), KK::LDS_BYTES, s, a);
}

template <typename TS, int R, int TBMAX, int VX, int K, int NW, bool PER, bool FAST, bool LATE, bool YL, bool FLX>
constexpr int lds_of() { return Kern<TS, R, TBMAX, VX, K, NW, PER, FAST, LATE, YL, FLX>::LDS_BYTES; }

template <typename TS, int R, int TBMAX, int VX, int K, int NW, bool PER, bool FAST, bool LATE, bool YL, bool FLX>
int occ_of() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, stream3d_kernel<TS, R, TBMAX, VX, K, NW, PER, FAST, LATE, YL, FLX>,
                                                     64 * NW,
                                                     lds_of<TS, R, TBMAX, VX, K, NW, PER, FAST, LATE, YL, FLX>()) != hipSuccess)
        n = 0;
    return n;
}

template <typename TS> constexpr int32_t dtype_of();
template <> constexpr int32_t dtype_of<double>() { return kF64; }
template <> constexpr int32_t dtype_of<float>() { return kF32; }
template <> constexpr int32_t dtype_of<bf16s>() { return kBF16; }

#define S3D_ENTRY(TS, R, TBM, VX, K, NW, PER, FAST, LATE, YL, FLX)                                        \
    Entry3{Stream3DKey{dtype_of<TS>(), (PER) ? kPeriodic : kZero, R, TBM, VX, K, NW, FAST, LATE, YL, FLX},    \
           &launch<TS, R, TBM, VX, K, NW, PER, FAST, LATE, YL, FLX>,                                                 \
           lds_of<TS, R, TBM, VX, K, NW, PER, FAST, LATE, YL, FLX>(), &occ_of<TS, R, TBM, VX, K, NW, PER, FAST, LATE, YL, FLX>}
#define S3D_BCLY(TS, R, TBM, VX, K, NW, LATE, YL)                                                      \
    S3D_ENTRY(TS, R, TBM, VX, K, NW, false, true, LATE, YL, false),                                    \
        S3D_ENTRY(TS, R, TBM, VX, K, NW, true, true, LATE, YL, false),                                 \
        S3D_ENTRY(TS, R, TBM, VX, K, NW, false, false, LATE, YL, false),                               \
        S3D_ENTRY(TS, R, TBM, VX, K, NW, true, false, LATE, YL, false)
#define S3D_BCL(TS, R, TBM, VX, K, NW, LATE) S3D_BCLY(TS, R, TBM, VX, K, NW, LATE, false)
#define S3D_BC(TS, R, TBM, VX, K, NW) S3D_BCL(TS, R, TBM, VX, K, NW, false)
#define S3D_BCY(TS, R, TBM, VX, K, NW, LATE) S3D_BCLY(TS, R, TBM, VX, K, NW, LATE, true)
// outflow-summing variants: zero rule only (the periodic grid has no boundary)
#define S3D_FLUX(TS, R, TBM, VX, K, NW, LATE, YL)                                                      \
    S3D_ENTRY(TS, R, TBM, VX, K, NW, false, true, LATE, YL, true),                                     \
        S3D_ENTRY(TS, R, TBM, VX, K, NW, false, false, LATE, YL, true)

}  // namespace s3d
}  // namespace st
