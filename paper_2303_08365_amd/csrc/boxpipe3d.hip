// boxpipe3d.hip -- 3D radius-1 boxes (27 points), two steps fused per pass,
// the z direction kept as partial sums, one LDS row exchange per plane.
//
// Tiling as in the other 2.5-D kernels (paper Sec. 4.1: an xy tile held on
// chip while the work-group streams along z; Sec. 4.2: tiles staged on chip
// so global accesses stay coalesced): lane L of wave w holds columns
// X0 + L*VX .. +VX-1 of rows Y0 + w*K .. +K-1.  x neighbours come from the
// lane's own registers or lane +-1 through DPP (0 enters at the register
// tile's edges), y neighbours from the wave's own rows or the row just above
// and below it.
//
// Canonical point order of a box: the centre, then (dz, dy, dx)
// lexicographic, one multiply and an FMA chain.  The chain of plane z takes
// plane z-1's nine points before plane z's and plane z+1's last, so a level
// keeps, besides its previous plane, the partial sum P(z-1) =
// centre + plane z-2 + plane z-1 of its next plane; when its plane z
// arrives with its neighbour rows, the nine terms of plane z finish
// u_{l+1}(z-1), and P(z) is started: centre of plane z, the nine terms of
// plane z-1, the eight other terms of plane z.  Same operations in the same
// order as the one-step kernel, so both give the same bits.
//
// Level 0's plane arrives from HBM with the rows just above and below the
// wave (other waves' rows, from L2), so level 1 is exact on the whole tile.
// Level 1's new plane goes to level 2 in the NEXT iteration: its first and
// last rows are written to an LDS buffer, and after the barrier that opens
// the next iteration every wave reads its row above and below from there.
// Two buffers alternate by iteration, so one barrier per plane suffices;
// the tile's halo rows at level 1 are LDS rows that stay 0.  Level 2 is
// therefore exact on the tile shrunk by one row and two columns per side;
// under the zero rule a tile that would cross the grid edge is moved inward
// to touch it, where the zeros are the ghost layer.  Level 1's ghost planes
// are set to 0 explicitly (one select per value).
//
// Memory access: one buffer descriptor per plane (empty for a ghost plane)
// and a 32-bit vector offset per row fixed for the pass; rows outside the
// grid and cells the tile does not own use an offset past the range, so
// such loads return 0 and such stores are dropped.  Needs the zero rule,
// nx >= 64*VX, ny >= NW*K, planes below 2 GiB and, for an even VX,
// nx % VX == 0.
#include "dev_common.h"
#include "internal.h"

namespace st {
namespace bp3d {

// PR: level 0 and the LDS write of its plane's edge rows -- what the other
// waves wait for at the next barrier -- run at wave priority 1.
template <typename TS, int VX, int K, int NW, bool PR = false>
struct Pipe {
    using S = Storage<TS>;
    using TC = typename S::TC;
    static constexpr int W = 64 * VX;
    static constexpr int H = NW * K;
    static constexpr int R = K + 2;                      // a wave's rows with the rows above and below
    static constexpr int HXA = (2 + VX - 1) / VX * VX;   // inexact columns per side after two steps, whole lanes
    static constexpr int OUTW = W - 2 * HXA;
    static constexpr int OUTH = H - 2;
    // LDS rows of one buffer: slot 0 the zero row above the tile, 2w+1 and
    // 2w+2 the first and last row of wave w, 2*NW+1 the zero row below.
    // Wave w reads its row above from slot 2w and its row below from 2w+3.
    static constexpr int SLOTS = 2 * NW + 2;
    static constexpr int BUF = SLOTS * W;
    static constexpr uint32_t kOut = 0x80000000u;       // past the end of any plane (planes < 2 GiB)
    static constexpr int32_t kRsrcWord3 = 0x00020000;  // gfx9: raw 32-bit data
    static constexpr int kNT = 2;                      // stores: non-temporal
    // An odd lane width cannot keep tile edges on lane boundaries (the edge
    // tiles touch the grid's edge): then ownership and stores go per element.
    static constexpr bool kElem = VX % 2 != 0;
    static constexpr int SO = kElem ? K * VX : K;

    struct Ctx {
        const TS* src;
        TS* dst;
        int32_t nz, zs, ze;
        int64_t plane_elems;
        uint32_t plane_bytes;
        uint32_t lo[R];  // byte offset of the lane's columns in rows yw-1 .. yw+K; kOut outside the grid
        uint32_t so[SO];  // same for the stores of the wave's rows (per element if kElem); kOut: not owned
        int lane, wave;
        TC w[27];
    };

    // a wave-uniform weight in scalar registers
    static __device__ __forceinline__ TC suni(TC v) {
        if constexpr (sizeof(TC) == 8) return uni(v);
        else return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
    }
    static __device__ __forceinline__ bool zghost(int32_t z, int32_t nz) {
        return static_cast<uint32_t>(z) >= static_cast<uint32_t>(nz);
    }
    static __device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_in(const Ctx& c, int32_t z) {
        const bool out = zghost(z, c.nz);
        const TS* base = out ? c.src : c.src + static_cast<int64_t>(z) * c.plane_elems;
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<TS*>(base), 0, out ? 0 : c.plane_bytes, kRsrcWord3);
    }
    static __device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_out(const Ctx& c, int32_t z) {
        const bool ok = static_cast<uint32_t>(z - c.zs) < static_cast<uint32_t>(c.ze - c.zs);
        TS* base = ok ? c.dst + static_cast<int64_t>(z) * c.plane_elems : c.dst;
        return __builtin_amdgcn_make_buffer_rsrc(base, 0, ok ? c.plane_bytes : 0, kRsrcWord3);
    }

    static __device__ __forceinline__ void ldrow(__amdgpu_buffer_rsrc_t r, uint32_t vo, TC (&v)[VX]) {
        constexpr int kBytes = VX * static_cast<int>(sizeof(TS));
        static_assert(kBytes == 8 || kBytes % 8 == 0, "rows are read in 8- or 16-byte pieces");
        TS vals[VX];
        if constexpr (kBytes % 16 == 0) {
            u32x4 raw[kBytes / 16];
#pragma unroll
            for (int i = 0; i < kBytes / 16; ++i)
                raw[i] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(r, vo + 16 * i, 0, 0));
            __builtin_memcpy(vals, raw, kBytes);
        } else if constexpr (kBytes > 16) {
            u32x2 raw[kBytes / 8];
#pragma unroll
            for (int i = 0; i < kBytes / 16; ++i) {
                const u32x4 q = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(r, vo + 16 * i, 0, 0));
                raw[2 * i] = u32x2{q[0], q[1]};
                raw[2 * i + 1] = u32x2{q[2], q[3]};
            }
            raw[kBytes / 8 - 1] =
                __builtin_bit_cast(u32x2, __builtin_amdgcn_raw_buffer_load_b64(r, vo + kBytes - 8, 0, 0));
            __builtin_memcpy(vals, raw, kBytes);
        } else {
            const u32x2 raw = __builtin_bit_cast(u32x2, __builtin_amdgcn_raw_buffer_load_b64(r, vo, 0, 0));
            __builtin_memcpy(vals, &raw, kBytes);
        }
#pragma unroll
        for (int e = 0; e < VX; ++e) v[e] = S::widen(vals[e]);
    }
    static __device__ __forceinline__ void strow(__amdgpu_buffer_rsrc_t r, uint32_t vo, const TC (&v)[VX]) {
        constexpr int kBytes = VX * static_cast<int>(sizeof(TS));
        TS vals[VX];
#pragma unroll
        for (int e = 0; e < VX; ++e) vals[e] = S::narrow(v[e]);
        if constexpr (kBytes % 16 == 0) {
            u32x4 raw[kBytes / 16];
            __builtin_memcpy(raw, vals, kBytes);
#pragma unroll
            for (int i = 0; i < kBytes / 16; ++i) __builtin_amdgcn_raw_buffer_store_b128(raw[i], r, vo + 16 * i, 0, kNT);
        } else if constexpr (kBytes > 16) {
            u32x2 raw[kBytes / 8];
            __builtin_memcpy(raw, vals, kBytes);
#pragma unroll
            for (int i = 0; i < kBytes / 16; ++i)
                __builtin_amdgcn_raw_buffer_store_b128(u32x4{raw[2 * i][0], raw[2 * i][1], raw[2 * i + 1][0], raw[2 * i + 1][1]},
                                                       r, vo + 16 * i, 0, kNT);
            __builtin_amdgcn_raw_buffer_store_b64(raw[kBytes / 8 - 1], r, vo + kBytes - 8, 0, kNT);
        } else {
            u32x2 raw;
            __builtin_memcpy(&raw, vals, kBytes);
            __builtin_amdgcn_raw_buffer_store_b64(raw, r, vo, 0, kNT);
        }
    }

    static __device__ __forceinline__ void load_plane(const Ctx& c, int32_t z, TC (&v)[R][VX]) {
        const __amdgpu_buffer_rsrc_t r = plane_in(c, z);
#pragma unroll
        for (int i = 0; i < R; ++i) ldrow(r, c.lo[i], v[i]);
    }
    static __device__ __forceinline__ void store_plane(const Ctx& c, int32_t z, const TC (&v)[K][VX]) {
        const __amdgpu_buffer_rsrc_t r = plane_out(c, z);
        if constexpr (kElem) {
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int e = 0; e < VX; ++e) {
                    const TS x = S::narrow(v[k][e]);
                    if constexpr (sizeof(TS) == 8)
                        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, c.so[k * VX + e], 0, kNT);
                    else if constexpr (sizeof(TS) == 4)
                        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, x), r, c.so[k * VX + e], 0, kNT);
                    else
                        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, x), r, c.so[k * VX + e], 0, kNT);
                }
        } else {
#pragma unroll
            for (int k = 0; k < K; ++k) strow(r, c.so[k], v[k]);
        }
    }

    // The value left of a row's first column and right of its last.
    static __device__ __forceinline__ void xnb(const TC (&v)[VX], TC& l, TC& r) {
        l = from_lower_z(v[VX - 1]);
        r = from_upper_z(v[0]);
    }
    static __device__ __forceinline__ TC at(const TC (&v)[VX], TC l, TC r, int x) {
        return x < 0 ? l : (x >= VX ? r : v[x < 0 ? 0 : (x >= VX ? 0 : x)]);
    }

    // acc += one plane's points in (dy, dx) order, weights from p0 on; the
    // plane's own centre is left out when SKIPC.
    template <bool SKIPC>
    static __device__ __forceinline__ void plane_terms(const Ctx& c, int p0, const TC (&u)[R][VX], const TC (&l)[R],
                                                       const TC (&r)[R], TC (&acc)[K][VX]) {
        int p = p0;
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                if (SKIPC && dy == 0 && dx == 0) continue;
#pragma unroll
                for (int k = 0; k < K; ++k)
#pragma unroll
                    for (int e = 0; e < VX; ++e)
                        acc[k][e] = fma_c(c.w[p], at(u[k + 1 + dy], l[k + 1 + dy], r[k + 1 + dy], e + dx), acc[k][e]);
                ++p;
            }
    }

    // One level: u = its plane z (with the rows above and below), prev its
    // plane z-1, P the partial sum of the next level's plane z-1.  out gets
    // the next level's plane z-1; P becomes the partial sum of plane z and
    // prev becomes u.  (The new partial sum's plane z-1 terms come first, so
    // the x neighbours of prev and of u are never held together.)
    static __device__ __forceinline__ void level(const Ctx& c, const TC (&u)[R][VX], TC (&prev)[R][VX], TC (&P)[K][VX],
                                                 TC (&out)[K][VX]) {
        TC Pn[K][VX];
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int e = 0; e < VX; ++e) Pn[k][e] = c.w[0] * u[k + 1][e];
        {
            TC pl[R], pr[R];
#pragma unroll
            for (int i = 0; i < R; ++i) xnb(prev[i], pl[i], pr[i]);
            plane_terms<false>(c, 1, prev, pl, pr, Pn);
        }
        TC ul[R], ur[R];
#pragma unroll
        for (int i = 0; i < R; ++i) xnb(u[i], ul[i], ur[i]);
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int e = 0; e < VX; ++e) out[k][e] = P[k][e];
        plane_terms<false>(c, 18, u, ul, ur, out);
        plane_terms<true>(c, 10, u, ul, ur, Pn);
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int e = 0; e < VX; ++e) P[k][e] = Pn[k][e];
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
            for (int e = 0; e < VX; ++e) prev[i][e] = u[i][e];
    }

    static __device__ __forceinline__ void run(const Box3DArgs& a, TC* lds) {
        Ctx c;
        c.lane = threadIdx.x & 63;
        c.wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
        const uint32_t tiles = static_cast<uint32_t>(a.tiles_x) * a.tiles_y * a.chunks_z;
        const uint32_t item = static_cast<uint32_t>(xcd_remap(blockIdx.x, gridDim.x));
        if (item >= tiles) return;
        const uint32_t txy = item / static_cast<uint32_t>(a.tiles_x);
        const int32_t tx = static_cast<int32_t>(item - txy * a.tiles_x);
        const int32_t ty = static_cast<int32_t>(txy % static_cast<uint32_t>(a.tiles_y));
        const int32_t cz = static_cast<int32_t>(txy / static_cast<uint32_t>(a.tiles_y));
        const int32_t nz = static_cast<int32_t>(a.nz), ny = static_cast<int32_t>(a.ny), nx = static_cast<int32_t>(a.nx);
        c.src = static_cast<const TS*>(a.src);
        c.dst = static_cast<TS*>(a.dst);
        c.nz = nz;
        c.plane_elems = static_cast<int64_t>(ny) * nx;
        c.plane_bytes = static_cast<uint32_t>(c.plane_elems * static_cast<int64_t>(sizeof(TS)));
        c.zs = cz * a.chunk_z;
        c.ze = c.zs + a.chunk_z < nz ? c.zs + a.chunk_z : nz;
        // owned cells and the register tile, moved inward at the grid edges
        const int32_t ox0 = tx * OUTW, ox1 = ox0 + OUTW < nx ? ox0 + OUTW : nx;
        const int32_t oy0 = ty * OUTH, oy1 = oy0 + OUTH < ny ? oy0 + OUTH : ny;
        int32_t X0 = ox0 - HXA;
        X0 = X0 < 0 ? 0 : (X0 + W > nx ? nx - W : X0);
        int32_t Y0 = oy0 - 1;
        Y0 = Y0 < 0 ? 0 : (Y0 + H > ny ? ny - H : Y0);
        const int32_t xl = X0 + c.lane * VX;
        const int32_t yw = Y0 + c.wave * K;
        constexpr uint32_t kE = static_cast<uint32_t>(sizeof(TS));
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int32_t y = yw - 1 + i;
            c.lo[i] = static_cast<uint32_t>(y) < static_cast<uint32_t>(ny)
                          ? static_cast<uint32_t>(y * nx + xl) * kE
                          : kOut;
        }
        if constexpr (kElem) {
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int e = 0; e < VX; ++e) {
                    const int32_t y = yw + k, x = xl + e;
                    c.so[k * VX + e] = x >= ox0 && x < ox1 && y >= oy0 && y < oy1
                                           ? static_cast<uint32_t>(y * nx + x) * kE
                                           : kOut;
                }
        } else {
            const bool xown = xl >= ox0 && xl + VX <= ox1;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int32_t y = yw + k;
                c.so[k] = xown && y >= oy0 && y < oy1 ? static_cast<uint32_t>(y * nx + xl) * kE : kOut;
            }
        }
#pragma unroll
        for (int p = 0; p < 27; ++p) c.w[p] = suni(static_cast<TC>(a.w[p]));

        // both exchange buffers start at 0 (the zero rows are never written)
        for (int i = static_cast<int>(threadIdx.x); i < 2 * BUF; i += 64 * NW) lds[i] = TC(0);

        TC pf[R][VX], u0p[R][VX], P0[K][VX], x1[K][VX], u1p[R][VX], P1[K][VX];
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
            for (int e = 0; e < VX; ++e) u0p[i][e] = u1p[i][e] = TC(0);
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int e = 0; e < VX; ++e) P0[k][e] = x1[k][e] = P1[k][e] = TC(0);

        // input planes zs-2 .. ze+2: the plane taken in iteration zin
        // finishes level 1's plane zin-1 and level 2's plane zin-3
        const int32_t zfirst = c.zs - 2, nit = c.ze - c.zs + 5;
        const int rd = 2 * c.wave * W + c.lane * VX;  // this lane's place in slot 2w
        load_plane(c, zfirst, pf);
        for (int32_t it = 0; it < nit; ++it) {
            const int32_t zin = zfirst + it;
            __syncthreads();
            if constexpr (PR) __builtin_amdgcn_s_setprio(1);
            TC u0[R][VX];
#pragma unroll
            for (int i = 0; i < R; ++i)
#pragma unroll
                for (int e = 0; e < VX; ++e) u0[i][e] = pf[i][e];
            load_plane(c, zin + 1, pf);
            // level 1's plane from the previous iteration, with the rows
            // above and below from the neighbouring waves
            TC u1[R][VX];
            const TC* rb = lds + ((it + 1) & 1) * BUF + rd;
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                u1[0][e] = rb[e];
                u1[R - 1][e] = rb[3 * W + e];
            }
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int e = 0; e < VX; ++e) u1[k + 1][e] = x1[k][e];
            TC o0[K][VX];
            level(c, u0, u0p, P0, o0);
            const bool g = zghost(zin - 1, nz);
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int e = 0; e < VX; ++e) x1[k][e] = g ? TC(0) : S::round(o0[k][e]);
            TC* wb = lds + (it & 1) * BUF + rd;
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                wb[W + e] = x1[0][e];
                wb[2 * W + e] = x1[K - 1][e];
            }
            if constexpr (PR) __builtin_amdgcn_s_setprio(0);
            TC o1[K][VX];
            level(c, u1, u1p, P1, o1);
            store_plane(c, zin - 3, o1);
        }
    }
};

template <typename TS, int VX, int K, int NW, bool PR = false>
__global__ __launch_bounds__(64 * NW) void boxpipe3d_kernel(const Box3DArgs a) {
    using P = Pipe<TS, VX, K, NW, PR>;
    __shared__ __align__(16) typename P::TC lds[2 * P::BUF];
    P::run(a, lds);
}

template <typename TS, int VX, int K, int NW, bool PR = false>
hipError_t launch_t(const Box3DArgs& a, hipStream_t s) {
    const int64_t tiles = static_cast<int64_t>(a.tiles_x) * a.tiles_y * a.chunks_z;
    hipLaunchKernelGGL((boxpipe3d_kernel<TS, VX, K, NW, PR>), dim3(static_cast<unsigned>(tiles)), dim3(64 * NW), 0, s, a);
    return hipGetLastError();
}

template <typename TS, int VX, int K, int NW, bool PR = false>
constexpr BoxPipeShape shape_t() {
    using P = Pipe<TS, VX, K, NW, PR>;
    return BoxPipeShape{VX, K, P::W, P::H, P::OUTW, P::OUTH, 64 * NW};
}

}  // namespace bp3d

// Instances per type (columns x rows a lane, 8 waves): FP64 2 x 3 (level 0
// at wave priority 1: 476 against 472 Gcell/s at 512^3) and 3 x 2 (2 x 4 and
// 3 x 3 spill), FP32 2 x 6, bfloat16 4 x 4.
int boxpipe3d_variants(int dtype) { return dtype == kF64 ? 2 : (dtype == kF32 || dtype == kBF16 ? 1 : 0); }

BoxPipeShape boxpipe3d_shape(int dtype, int v) {
    switch (dtype) {
        case kF64: return v == 0 ? bp3d::shape_t<double, 2, 3, 8, true>() : bp3d::shape_t<double, 3, 2, 8>();
        case kF32: return bp3d::shape_t<float, 2, 6, 8>();
        default: return bp3d::shape_t<bf16s, 4, 4, 8>();
    }
}

hipError_t launch_boxpipe3d(int dtype, int v, const Box3DArgs& a, hipStream_t s) {
    if (static_cast<int64_t>(a.tiles_x) * a.tiles_y * a.chunks_z <= 0) return hipSuccess;
    switch (dtype) {
        case kF64: return v == 0 ? bp3d::launch_t<double, 2, 3, 8, true>(a, s) : bp3d::launch_t<double, 3, 2, 8>(a, s);
        case kF32: return bp3d::launch_t<float, 2, 6, 8>(a, s);
        case kBF16: return bp3d::launch_t<bf16s, 4, 4, 8>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace st
