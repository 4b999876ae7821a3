// stream3d_impl.h -- 3D star stencils (radius R) with T_b steps fused per pass.
//
// 2.5-D blocking: an xy tile is held on chip while the work-group streams
// along z (paper Sec. 4.1 builds space-time tiles, tetrahedra in 3D; Sec. 4.2
// stages tiles on chip so global accesses stay coalesced).  On gfx950 the
// on-chip tile lives mostly in VGPRs:
//   * lane L of wave w holds columns X0 + L*VX .. +VX-1 of rows
//     Y0 + w*K .. Y0 + w*K + K-1 of every plane (one 16-byte access per row);
//   * pipeline level l keeps the last 2R+1 planes of step l (its z queue);
//   * x neighbours: own registers, or lane +-1 through DPP (the outermost R
//     columns of step 0 are loaded by lanes 0 and 63 and enter through the
//     DPP "old" operand);
//   * y neighbours: own rows, or the R edge rows of the wave above / below,
//     exchanged through LDS once per level and plane (the R rows above and
//     below the whole tile, for step 0, are loaded by the first / last wave);
//   * z neighbours: queue slots.
// Step l is exact on the register tile shrunk by (l-1)*R on each side; the
// tile interior [X0+hxa, X0+W-hxa) x [Y0+hya, Y0+H-hya), hxa, hya >=
// R*(tb-1), is stored.  A z chunk [zs, ze) loads planes zs-R*tb .. ze-1+R*tb.
//
// LDS (per buffer, two buffers alternate between barriers): tile rows
// -R .. H+R-1 of the plane being advanced; each wave publishes only the rows
// other waves read (its first R and last R rows), and the first / last wave
// the ring rows.
#pragma once

#include <utility>

#include "dev_common.h"
#include "registry.h"

namespace st {

namespace s3d {

template <typename TS, int R, int TBMAX, int VX, int K, int NW, bool PER>
struct Kern {
    using S = Storage<TS>;
    using TC = typename S::TC;
    static_assert(VX >= R, "a lane must hold at least R columns");
    static constexpr int Q = 2 * R + 1;
    static constexpr int W = 64 * VX;
    static constexpr int H = NW * K;
    static constexpr int NP = 6 * R + 1;
    // LDS row slot of tile row r (-R <= r < H + R) is r + R.
    static constexpr int SLOTS = H + 2 * R;
    static constexpr int BUF_ELEMS = SLOTS * W;
    static constexpr int LDS_BYTES = 2 * BUF_ELEMS * static_cast<int>(sizeof(TC));

    struct Ctx {
        const TS* src;
        TS* dst;
        int64_t nz, ny, nx;
        int64_t X0, Y0;
        int64_t xl;           // first column of this lane
        int64_t yw;           // first row of this wave
        int64_t zs, ze;
        int64_t ox0, ox1, oy0, oy1;   // output columns / rows
        bool fast;
        int lane, wave;
        TC w[NP];
    };

    static __device__ __forceinline__ int64_t plane_idx(const Ctx& c, int64_t z, bool& ghost) {
        ghost = false;
        if (z < 0 || z >= c.nz) {
            if (!PER) { ghost = true; return 0; }
            z = wrap_idx(z, c.nz);
        }
        return z;
    }

    // One row (x strip of this lane) of plane z, row y.
    static __device__ __forceinline__ void load_row(const Ctx& c, int64_t z, bool zghost, int64_t y,
                                                    TC (&v)[VX]) {
        bool ghost = zghost;
        if (y < 0 || y >= c.ny) {
            if (!PER) ghost = true; else y = wrap_idx(y, c.ny);
        }
        if (ghost) {
#pragma unroll
            for (int e = 0; e < VX; ++e) v[e] = TC(0);
            return;
        }
        const TS* row = c.src + (z * c.ny + y) * c.nx;
        if (c.fast) {
            ldv<TS, VX>(row + c.xl, v);
        } else {
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                const int64_t x = c.xl + e;
                if (PER) v[e] = ld1(row + wrap_idx(x, c.nx));
                else v[e] = (x >= 0 && x < c.nx) ? ld1(row + x) : TC(0);
            }
        }
    }

    static __device__ __forceinline__ void load_plane(const Ctx& c, int64_t z, TC (&v)[K][VX]) {
        bool zg;
        const int64_t zz = plane_idx(c, z, zg);
#pragma unroll
        for (int k = 0; k < K; ++k) load_row(c, zz, zg, c.yw + k, v[k]);
    }

    // x ring (lanes 0 and 63) for this wave's rows of plane z.
    static __device__ __forceinline__ void load_xring(const Ctx& c, int64_t z, TC (&r)[K][R]) {
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int j = 0; j < R; ++j) r[k][j] = TC(0);
        if (c.lane != 0 && c.lane != 63) return;
        bool zg;
        const int64_t zz = plane_idx(c, z, zg);
        if (zg) return;
        const int64_t xb = (c.lane == 0) ? c.X0 - R : c.X0 + W;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            int64_t y = c.yw + k;
            if (y < 0 || y >= c.ny) {
                if (!PER) continue;
                y = wrap_idx(y, c.ny);
            }
            const TS* row = c.src + (zz * c.ny + y) * c.nx;
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int64_t x = xb + j;
                if (PER) r[k][j] = ld1(row + wrap_idx(x, c.nx));
                else r[k][j] = (x >= 0 && x < c.nx) ? ld1(row + x) : TC(0);
            }
        }
    }

    // y ring: R rows above the tile (first wave) or below it (last wave).
    static __device__ __forceinline__ void load_yring(const Ctx& c, int64_t z, TC (&top)[R][VX],
                                                      TC (&bot)[R][VX]) {
        bool zg;
        const int64_t zz = plane_idx(c, z, zg);
        if (c.wave == 0) {
#pragma unroll
            for (int j = 0; j < R; ++j) load_row(c, zz, zg, c.Y0 - R + j, top[j]);
        }
        if (c.wave == NW - 1) {
#pragma unroll
            for (int j = 0; j < R; ++j) load_row(c, zz, zg, c.Y0 + H + j, bot[j]);
        }
    }

    static __device__ __forceinline__ void lds_put(TC* buf, int slot, int lane, const TC (&v)[VX]) {
        TC* p = buf + slot * W + lane * VX;
#pragma unroll
        for (int e = 0; e < VX; ++e) p[e] = v[e];
    }
    static __device__ __forceinline__ void lds_get(const TC* buf, int slot, int lane, TC (&v)[VX]) {
        const TC* p = buf + slot * W + lane * VX;
#pragma unroll
        for (int e = 0; e < VX; ++e) v[e] = p[e];
    }

    static __device__ __forceinline__ TC xval(const TC (&v)[VX], const TC (&lft)[R],
                                              const TC (&rgt)[R], int idx) {
        return idx < 0 ? lft[R + idx] : (idx >= VX ? rgt[idx - VX] : v[idx]);
    }

    // Step l+1 on plane (newest - R) from the queue of step l.  Canonical point
    // order for a 3D star: centre; z -R..-1; y -R..-1; x -R..-1; x +1..+R;
    // y +1..+R; z +1..+R.
    template <int J>
    static __device__ __forceinline__ void compute(const Ctx& c, const TC (&q)[Q][K][VX],
                                                   const TC (&xr)[K][R], const TC (&above)[R][VX],
                                                   const TC (&below)[R][VX], TC (&out)[K][VX]) {
        constexpr int CEN = (J - R + Q) % Q;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            TC lft[R], rgt[R];
#pragma unroll
            for (int j = 0; j < R; ++j) {
                lft[j] = from_lower(q[CEN][k][VX - R + j], xr[k][j]);
                rgt[j] = from_upper(q[CEN][k][j], xr[k][j]);
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

    static __device__ __forceinline__ void finish(const Ctx& c, int64_t z, TC (&out)[K][VX]) {
        if (!PER) {
            const bool zg = z < 0 || z >= c.nz;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int64_t y = c.yw + k;
                const bool rowg = zg || y < 0 || y >= c.ny;
#pragma unroll
                for (int e = 0; e < VX; ++e) {
                    const int64_t x = c.xl + e;
                    if (rowg || (!c.fast && (x < 0 || x >= c.nx))) out[k][e] = TC(0);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int e = 0; e < VX; ++e) out[k][e] = S::round(out[k][e]);
    }

    static __device__ __forceinline__ void store_plane(const Ctx& c, int64_t z, const TC (&out)[K][VX]) {
        if (z < c.zs || z >= c.ze) return;
        if (c.xl < c.ox0 || c.xl >= c.ox1) return;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int64_t y = c.yw + k;
            if (y < c.oy0 || y >= c.oy1 || y >= c.ny) continue;
            TS* row = c.dst + (z * c.ny + y) * c.nx;
            if (c.fast) {
                stv<TS, VX>(row + c.xl, out[k]);
            } else {
#pragma unroll
                for (int e = 0; e < VX; ++e) {
                    const int64_t x = c.xl + e;
                    if (x < c.nx) st1(row + x, out[k][e]);
                }
            }
        }
    }

    struct State {
        TC q[TBMAX][Q][K][VX];
        TC pf[K][VX];
        TC xr[K][R], nxr[K][R];
        TC top[R][VX], bot[R][VX], ntop[R][VX], nbot[R][VX];
    };

    template <int J>
    static __device__ __forceinline__ void step(const Ctx& c, int tb, int64_t it, int64_t nit,
                                                int64_t zfirst, State& s, TC* lds) {
        const int64_t zin = zfirst + it;
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int e = 0; e < VX; ++e) s.q[0][J][k][e] = s.pf[k][e];
        // rings of the step-0 centre plane (zin - R) were fetched last iteration
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int j = 0; j < R; ++j) s.xr[k][j] = s.nxr[k][j];
#pragma unroll
        for (int j = 0; j < R; ++j)
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                s.top[j][e] = s.ntop[j][e];
                s.bot[j][e] = s.nbot[j][e];
            }
        if (it + 1 < nit) {
            load_plane(c, zin + 1, s.pf);
            load_xring(c, zin + 1 - R, s.nxr);
            load_yring(c, zin + 1 - R, s.ntop, s.nbot);
        }
        constexpr int CEN = (J - R + Q) % Q;
#pragma unroll
        for (int l = 0; l < TBMAX; ++l) {
            if (l < tb) {
                TC* buf = lds + ((it * tb + l) & 1) * BUF_ELEMS;
                // publish the rows of the centre plane that other waves read
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    if (k < R || k >= K - R) lds_put(buf, c.wave * K + k + R, c.lane, s.q[l][CEN][k]);
                }
                if (l == 0) {
                    if (c.wave == 0) {
#pragma unroll
                        for (int j = 0; j < R; ++j) lds_put(buf, j, c.lane, s.top[j]);
                    }
                    if (c.wave == NW - 1) {
#pragma unroll
                        for (int j = 0; j < R; ++j) lds_put(buf, H + R + j, c.lane, s.bot[j]);
                    }
                }
                __syncthreads();
                TC above[R][VX], below[R][VX];
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    lds_get(buf, c.wave * K + j, c.lane, above[j]);          // row wK - R + j
                    lds_get(buf, c.wave * K + K + R + j, c.lane, below[j]);  // row wK + K + j
                }
                TC out[K][VX];
                if (l == 0) {
                    compute<J>(c, s.q[0], s.xr, above, below, out);
                } else {
                    TC zr[K][R];
#pragma unroll
                    for (int k = 0; k < K; ++k)
#pragma unroll
                        for (int j = 0; j < R; ++j) zr[k][j] = TC(0);
                    compute<J>(c, s.q[l], zr, above, below, out);
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
    static __device__ __forceinline__ void unroll_steps(const Ctx& c, int tb, int64_t base, int64_t nit,
                                                        int64_t zfirst, State& s, TC* lds,
                                                        std::integer_sequence<int, J...>) {
        ((base + J < nit ? step<J>(c, tb, base + J, nit, zfirst, s, lds) : void()), ...);
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
        c.src = static_cast<const TS*>(a.src);
        c.dst = static_cast<TS*>(a.dst);
        c.nz = a.nz;
        c.ny = a.ny;
        c.nx = a.nx;
        c.X0 = tx * a.out_w - a.hxa;
        c.Y0 = ty * a.out_h - a.hya;
        c.xl = c.X0 + static_cast<int64_t>(c.lane) * VX;
        c.yw = c.Y0 + static_cast<int64_t>(c.wave) * K;
        c.zs = cz * a.chunk_z;
        c.ze = c.zs + a.chunk_z < c.nz ? c.zs + a.chunk_z : c.nz;
        c.ox0 = c.X0 + a.hxa;
        c.ox1 = c.ox0 + a.out_w;
        c.oy0 = c.Y0 + a.hya;
        c.oy1 = c.oy0 + a.out_h;
        c.fast = a.vec_ok && c.X0 - R >= 0 && c.X0 + W + R <= c.nx && c.Y0 - R >= 0 &&
                 c.Y0 + H + R <= c.ny;
#pragma unroll
        for (int p = 0; p < NP; ++p) c.w[p] = static_cast<TC>(a.w[p]);
        const int tb = a.tb;
        const int64_t zfirst = c.zs - static_cast<int64_t>(R) * tb;
        const int64_t nit = (c.ze - c.zs) + 2 * static_cast<int64_t>(R) * tb;

        State s;
#pragma unroll
        for (int l = 0; l < TBMAX; ++l)
#pragma unroll
            for (int sl = 0; sl < Q; ++sl)
#pragma unroll
                for (int k = 0; k < K; ++k)
#pragma unroll
                    for (int e = 0; e < VX; ++e) s.q[l][sl][k][e] = TC(0);
#pragma unroll
        for (int j = 0; j < R; ++j)
#pragma unroll
            for (int e = 0; e < VX; ++e) s.ntop[j][e] = s.nbot[j][e] = TC(0);
        load_plane(c, zfirst, s.pf);
        load_xring(c, zfirst - R, s.nxr);
        load_yring(c, zfirst - R, s.ntop, s.nbot);
        for (int64_t base = 0; base < nit; base += Q)
            unroll_steps(c, tb, base, nit, zfirst, s, lds, std::make_integer_sequence<int, Q>{});
    }
};

template <typename TS, int R, int TBMAX, int VX, int K, int NW, bool PER>
__global__ __launch_bounds__(64 * NW) void stream3d_kernel(const Stream3DArgs a) {
    using KK = Kern<TS, R, TBMAX, VX, K, NW, PER>;
    extern __shared__ __align__(16) unsigned char smem[];
    KK::run(a, reinterpret_cast<typename KK::TC*>(smem));
}

using Launcher = void (*)(const Stream3DArgs&, hipStream_t);

template <typename TS, int R, int TBMAX, int VX, int K, int NW, bool PER>
void launch(const Stream3DArgs& a, hipStream_t s) {
    using KK = Kern<TS, R, TBMAX, VX, K, NW, PER>;
    const int64_t tiles = static_cast<int64_t>(a.tiles_x) * a.tiles_y * a.chunks_z;
    hipLaunchKernelGGL((stream3d_kernel<TS, R, TBMAX, VX, K, NW, PER>),
                       dim3(static_cast<unsigned>(tiles)), dim3(64 * NW), KK::LDS_BYTES, s, a);
}

template <typename TS, int R, int TBMAX, int VX, int K, int NW, bool PER>
constexpr int lds_of() { return Kern<TS, R, TBMAX, VX, K, NW, PER>::LDS_BYTES; }

template <typename TS> constexpr int32_t dtype_of();
template <> constexpr int32_t dtype_of<double>() { return kF64; }
template <> constexpr int32_t dtype_of<float>() { return kF32; }
template <> constexpr int32_t dtype_of<bf16s>() { return kBF16; }

#define S3D_ENTRY(TS, R, TBM, VX, K, NW, PER)                                              \
    Entry3{Stream3DKey{dtype_of<TS>(), (PER) ? kPeriodic : kZero, R, TBM, VX, K, NW},      \
           &launch<TS, R, TBM, VX, K, NW, PER>, lds_of<TS, R, TBM, VX, K, NW, PER>()}
#define S3D_BC(TS, R, TBM, VX, K, NW) \
    S3D_ENTRY(TS, R, TBM, VX, K, NW, false), S3D_ENTRY(TS, R, TBM, VX, K, NW, true)

}  // namespace s3d
}  // namespace st
