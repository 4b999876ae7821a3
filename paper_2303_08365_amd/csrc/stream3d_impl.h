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
// are unconditional: ghost cells (zero rule) are replaced by 0 with selects
// when the values are consumed, so no branch separates a load from its use
// and the prefetch stays in flight.
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

template <typename TS, int R, int TBMAX, int VX, int K, int NW, bool PER, bool FAST, bool LATE, bool YL>
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
        const ST_GLOBAL TS* src;
        ST_GLOBAL TS* dst;
        int64_t nz, ny, nx;
        int64_t X0, Y0;
        int64_t xl;            // first column of this lane
        int64_t yw;            // first row of this wave
        int64_t zs, ze, zlast; // output planes [zs, ze); last streamed plane
        int64_t ox0, ox1, oy0, oy1;
        int64_t xr_x, xr_y;    // the x-ring element this lane fetches
        int64_t hy[HR > 0 ? HR : 1];   // YL: grid rows of this wave's halo rows
        int hslot[HR > 0 ? HR : 1];    // YL: their LDS slots
        int lane, wave;
        TC w[NP];
    };

    // index rules: periodic wraps, zero clamps (the value is then masked)
    static __device__ __forceinline__ int64_t fix(int64_t i, int64_t n) {
        if (PER) return wrap_idx(i, n);
        return i < 0 ? 0 : (i >= n ? n - 1 : i);
    }
    static __device__ __forceinline__ bool ghost(int64_t i, int64_t n) {
        return !PER && (i < 0 || i >= n);
    }

    static __device__ __forceinline__ void load_row(const Ctx& c, int64_t zz, int64_t y, TC (&v)[VX]) {
        const ST_GLOBAL TS* row = c.src + (zz * c.ny + fix(y, c.ny)) * c.nx;
        if constexpr (FAST) {
            ldv<TS, VX>(row + (PER ? wrap_idx(c.xl, c.nx) : c.xl), v);
        } else {
#pragma unroll
            for (int e = 0; e < VX; ++e) v[e] = ld1(row + fix(c.xl + e, c.nx));
        }
    }

    // Loads of one pipeline slot: the wave's K rows of plane zm, and the ring
    // (2R rows, one x-ring value per lane) of plane zr.
    static __device__ __forceinline__ void load_main(const Ctx& c, int64_t zm, TC (&v)[K][VX]) {
        const int64_t zz = fix(zm < c.zlast ? zm : c.zlast, c.nz);
#pragma unroll
        for (int k = 0; k < K; ++k) load_row(c, zz, c.yw + k, v[k]);
    }
    static __device__ __forceinline__ void load_ring(const Ctx& c, int64_t zr, TC (&r)[RROWS][VX], TC& xv) {
        const int64_t zz = fix(zr < c.zlast ? zr : c.zlast, c.nz);
        if constexpr (YL) {
#pragma unroll
            for (int j = 0; j < HR; ++j) load_row(c, zz, c.hy[j], r[j]);
        } else {
#pragma unroll
            for (int j = 0; j < R; ++j) {
                load_row(c, zz, c.yw - R + j, r[j]);
                load_row(c, zz, c.yw + K + j, r[R + j]);
            }
        }
        xv = ld1(c.src + (zz * c.ny + fix(c.xr_y, c.ny)) * c.nx + fix(c.xr_x, c.nx));
    }

    // Ghost masks applied when a slot is consumed.
    static __device__ __forceinline__ void take_main(const Ctx& c, int64_t z, const TC (&v)[K][VX],
                                                     TC (&q)[K][VX]) {
        const bool zg = ghost(z, c.nz);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const bool rg = zg || (!FAST && ghost(c.yw + k, c.ny));
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                const bool g = rg || (!FAST && ghost(c.xl + e, c.nx));
                q[k][e] = g ? TC(0) : v[k][e];
            }
        }
    }
    static __device__ __forceinline__ void take_ring(const Ctx& c, int64_t z, const TC (&r)[RROWS][VX],
                                                     TC xv, TC (&above)[R][VX], TC (&below)[R][VX],
                                                     TC& xg) {
        static_assert(!YL, "the YL variants take their halo rows with take_halo");
        const bool zg = ghost(z, c.nz);
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const bool ga = zg || ghost(c.yw - R + j, c.ny);
            const bool gb = zg || ghost(c.yw + K + j, c.ny);
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                const bool xe = !FAST && ghost(c.xl + e, c.nx);
                above[j][e] = (ga || xe) ? TC(0) : r[j][e];
                below[j][e] = (gb || xe) ? TC(0) : r[R + j][e];
            }
        }
        xg = (zg || ghost(c.xr_y, c.ny) || ghost(c.xr_x, c.nx)) ? TC(0) : xv;
    }
    static __device__ __forceinline__ void take_halo(const Ctx& c, int64_t z, const TC (&r)[RROWS][VX],
                                                     TC xv, TC (&h)[RROWS][VX], TC& xg) {
        const bool zg = ghost(z, c.nz);
#pragma unroll
        for (int j = 0; j < RROWS; ++j) {
            const bool g = zg || ghost(c.hy[j], c.ny);
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                const bool xe = !FAST && ghost(c.xl + e, c.nx);
                h[j][e] = (g || xe) ? TC(0) : r[j][e];
            }
        }
        xg = (zg || ghost(c.xr_y, c.ny) || ghost(c.xr_x, c.nx)) ? TC(0) : xv;
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
                const TC ol = LEVEL0 ? lane_value(xg, k * R + j) : TC(0);
                const TC orr = LEVEL0 ? lane_value(xg, 32 + k * R + j) : TC(0);
                lft[j] = from_lower(q[CEN][k][VX - R + j], ol);
                rgt[j] = from_upper(q[CEN][k][j], orr);
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

    // Zero rule: ghost cells stay 0; bfloat16 storage rounds every step.
    static __device__ __forceinline__ void finish(const Ctx& c, int64_t z, TC (&out)[K][VX]) {
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

    static __device__ __forceinline__ void store_plane(const Ctx& c, int64_t z, const TC (&out)[K][VX]) {
        if (z < c.zs || z >= c.ze) return;
        if (c.xl < c.ox0 || c.xl >= c.ox1) return;  // lanes are wholly in or out
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int64_t y = c.yw + k;
            if (y < c.oy0 || y >= c.oy1) continue;
            ST_GLOBAL TS* row = c.dst + (z * c.ny + y) * c.nx;
            if constexpr (FAST) {
                stv<TS, VX>(row + c.xl, out[k]);
            } else {
#pragma unroll
                for (int e = 0; e < VX; ++e)
                    if (c.xl + e < c.nx) st1(row + c.xl + e, out[k][e]);
            }
        }
    }

    struct State {
        TC q[TBMAX][Q][K][VX];
        TC pf[LATE ? 1 : P][K][VX];  // unused when LATE
        TC rpf[PR][RROWS][VX];
        TC xpf[PR];
    };

    template <int J>
    static __device__ __forceinline__ void step(const Ctx& c, int tb, int64_t it, int64_t zfirst, State& s,
                                                TC* lds) {
        constexpr int SM = J % P, SR = J % PR;
        const int64_t zin = zfirst + it;
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

        constexpr int CEN = (J - R + Q) % Q;
#pragma unroll
        for (int l = 0; l < TBMAX; ++l) {
            if (l < tb) {
                TC out[K][VX];
                if (l == 0 && !YL) {
                    compute<J, true>(c, s.q[0], xg, above0, below0, out);
                } else {
                    // exchange the edge rows of this level's centre plane; with
                    // YL every level's exchange also fills the 2R halo slots
                    // (step 0: the loaded halo rows, later steps: 0)
                    const int64_t seq = YL ? it * tb + l : it * (tb - 1) + (l - 1);
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
                const int64_t zc = zin - static_cast<int64_t>(l + 1) * R;
                finish(c, zc, out);
                if (l + 1 == tb) {
                    store_plane(c, zc, out);
                } else if (l + 1 < TBMAX) {
#pragma unroll
                    for (int k = 0; k < K; ++k)
#pragma unroll
                        for (int e = 0; e < VX; ++e) s.q[l + 1][J][k][e] = out[k][e];
                }
            }
        }
    }

    template <int... J>
    static __device__ __forceinline__ void group(const Ctx& c, int tb, int64_t base, int64_t zfirst, State& s,
                                                 TC* lds, std::integer_sequence<int, J...>) {
        (step<J>(c, tb, base + J, zfirst, s, lds), ...);
    }
    template <int... J>
    static __device__ __forceinline__ void tail(const Ctx& c, int tb, int64_t base, int64_t nit, int64_t zfirst,
                                                State& s, TC* lds, std::integer_sequence<int, J...>) {
        ((base + J < nit ? step<J>(c, tb, base + J, zfirst, s, lds) : void()), ...);
    }

    static __device__ void run(const Stream3DArgs& a, TC* lds) {
        Ctx c;
        c.lane = threadIdx.x & 63;
        c.wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
        const int64_t tiles = static_cast<int64_t>(a.tiles_x) * a.tiles_y * a.chunks_z;
        const int64_t item = xcd_remap(blockIdx.x, gridDim.x);
        if (item >= tiles) return;
        const int64_t tx = item % a.tiles_x;
        const int64_t ty = (item / a.tiles_x) % a.tiles_y;
        const int64_t cz = item / (static_cast<int64_t>(a.tiles_x) * a.tiles_y);
        c.src = gptr<TS>(a.src);
        c.dst = gptr_mut<TS>(a.dst);
        c.nz = a.nz;
        c.ny = a.ny;
        c.nx = a.nx;
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
        c.xl = c.X0 + static_cast<int64_t>(c.lane) * VX;
        c.yw = c.Y0 + static_cast<int64_t>(c.wave) * K;
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
            }
        }
        c.zs = cz * a.chunk_z;
        c.ze = c.zs + a.chunk_z < c.nz ? c.zs + a.chunk_z : c.nz;
#pragma unroll
        for (int p = 0; p < NP; ++p) c.w[p] = static_cast<TC>(a.w[p]);
        const int tb = a.tb;
        const int64_t zfirst = c.zs - static_cast<int64_t>(R) * tb;
        const int64_t nit = (c.ze - c.zs) + 2 * static_cast<int64_t>(R) * tb;
        c.zlast = zfirst + nit - 1;

        if constexpr (TBMAX > 1 && !YL) {
            // ring rows of every LDS buffer stay 0 (ghost / unused halo)
            for (int i = threadIdx.x; i < 2 * R * W; i += blockDim.x) {
                const int row = i / W, col = i % W;
                const int slot = row < R ? row : H + row;
                lds[slot * W + col] = TC(0);
                lds[BUF_ELEMS + slot * W + col] = TC(0);
            }
            __syncthreads();
        }

        State s;
#pragma unroll
        for (int l = 0; l < TBMAX; ++l)
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

        int64_t base = 0;
        for (; base + Q <= nit; base += Q)
            group(c, tb, base, zfirst, s, lds, std::make_integer_sequence<int, Q>{});
        tail(c, tb, base, nit, zfirst, s, lds, std::make_integer_sequence<int, Q>{});
    }
};

template <typename TS, int R, int TBMAX, int VX, int K, int NW, bool PER, bool FAST, bool LATE, bool YL>
__global__ __launch_bounds__(64 * NW) void stream3d_kernel(const Stream3DArgs a) {
    using KK = Kern<TS, R, TBMAX, VX, K, NW, PER, FAST, LATE, YL>;
    extern __shared__ __align__(16) unsigned char smem[];
    KK::run(a, reinterpret_cast<typename KK::TC*>(smem));
}

template <typename TS, int R, int TBMAX, int VX, int K, int NW, bool PER, bool FAST, bool LATE, bool YL>
void launch(const Stream3DArgs& a, hipStream_t s) {
    using KK = Kern<TS, R, TBMAX, VX, K, NW, PER, FAST, LATE, YL>;
    const int64_t tiles = static_cast<int64_t>(a.tiles_x) * a.tiles_y * a.chunks_z;
    hipLaunchKernelGGL((stream3d_kernel<TS, R, TBMAX, VX, K, NW, PER, FAST, LATE, YL>),
                       dim3(static_cast<unsigned>(tiles)), dim3(64 * NW), KK::LDS_BYTES, s, a);
}

template <typename TS, int R, int TBMAX, int VX, int K, int NW, bool PER, bool FAST, bool LATE, bool YL>
constexpr int lds_of() { return Kern<TS, R, TBMAX, VX, K, NW, PER, FAST, LATE, YL>::LDS_BYTES; }

template <typename TS, int R, int TBMAX, int VX, int K, int NW, bool PER, bool FAST, bool LATE, bool YL>
int occ_of() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, stream3d_kernel<TS, R, TBMAX, VX, K, NW, PER, FAST, LATE, YL>,
                                                     64 * NW,
                                                     lds_of<TS, R, TBMAX, VX, K, NW, PER, FAST, LATE, YL>()) != hipSuccess)
        n = 0;
    return n;
}

template <typename TS> constexpr int32_t dtype_of();
template <> constexpr int32_t dtype_of<double>() { return kF64; }
template <> constexpr int32_t dtype_of<float>() { return kF32; }
template <> constexpr int32_t dtype_of<bf16s>() { return kBF16; }

#define S3D_ENTRY(TS, R, TBM, VX, K, NW, PER, FAST, LATE, YL)                                             \
    Entry3{Stream3DKey{dtype_of<TS>(), (PER) ? kPeriodic : kZero, R, TBM, VX, K, NW, FAST, LATE, YL},         \
           &launch<TS, R, TBM, VX, K, NW, PER, FAST, LATE, YL>,                                                 \
           lds_of<TS, R, TBM, VX, K, NW, PER, FAST, LATE, YL>(), &occ_of<TS, R, TBM, VX, K, NW, PER, FAST, LATE, YL>}
#define S3D_BCLY(TS, R, TBM, VX, K, NW, LATE, YL)                                                      \
    S3D_ENTRY(TS, R, TBM, VX, K, NW, false, true, LATE, YL), S3D_ENTRY(TS, R, TBM, VX, K, NW, true, true, LATE, YL), \
        S3D_ENTRY(TS, R, TBM, VX, K, NW, false, false, LATE, YL),                                      \
        S3D_ENTRY(TS, R, TBM, VX, K, NW, true, false, LATE, YL)
#define S3D_BCL(TS, R, TBM, VX, K, NW, LATE) S3D_BCLY(TS, R, TBM, VX, K, NW, LATE, false)
#define S3D_BC(TS, R, TBM, VX, K, NW) S3D_BCL(TS, R, TBM, VX, K, NW, false)
#define S3D_BCY(TS, R, TBM, VX, K, NW, LATE) S3D_BCLY(TS, R, TBM, VX, K, NW, LATE, true)

}  // namespace s3d
}  // namespace st
