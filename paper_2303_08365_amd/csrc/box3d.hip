// box3d.hip -- 3D radius-1 boxes (27 points), T_b = 1 or 2 steps per pass,
// planes streamed along z.
//
// 2.5-D blocking (paper Sec. 4.1 builds space-time tiles, Sec. 4.2 stages
// them on chip): a work-group holds an xy tile of 64*VX columns by NW*K rows
// and streams the planes of a z chunk; every wave works on its own.  Lane L
// of wave w holds columns X0 + L*VX .. + VX - 1 of its K rows plus T_b rows
// above and below (other waves' rows, loaded again from L2): step l (0-based)
// is computed on K + 2(T_b - 1 - l) rows, so the last step yields exactly the
// wave's K rows without any exchange between waves.  Each step keeps the last
// three planes of its input (its z queue).  x neighbours come from the
// neighbouring lanes by DPP; at step 0 the columns just outside the tile come
// from one load per plane (lanes 0.. fetch the left column of the rows,
// lanes 32.. the right one) and enter lane 0 / lane 63 as the DPP "old"
// operand through readlane; deeper steps lose one column per side, so tiles
// overlap by whole lanes (zero rule: the edge tiles move inward and the zero
// entering through DPP is the ghost cell).  Every load is a buffer load
// through a descriptor whose range is the row (the plane for the outer
// columns), empty outside the grid, so the zero rule's ghost cells load as 0;
// intermediate steps zero their ghost planes and rows explicitly.
//
// Canonical point order: centre, then (dz, dy, dx) lexicographic -- the
// one-step kernel's order, one multiply then an FMA chain, so all depths give
// the same bits.
#include "dev_common.h"

namespace st {
namespace b3d {

template <typename TS, int VX, int K, int NW, int TB, bool PER, bool FAST>
struct Kern {
    using S = Storage<TS>;
    using TC = typename S::TC;
    static constexpr int W = 64 * VX;
    static constexpr int H = NW * K;
    static constexpr int RIN = K + 2 * TB;                  // rows of the input planes
    static constexpr int HX = ((TB - 1) + VX - 1) / VX * VX;  // stale columns per tile side
    static_assert(RIN <= 32, "the outer columns of a wave's rows fit in half a wave");
    static constexpr int32_t kRsrcWord3 = 0x00020000;
    static constexpr int32_t kNT = 2;

    struct Ctx {
        const TS* src;
        TS* dst;
        int32_t nz, ny, nx;
        int64_t plane_elems;
        uint32_t row_bytes, plane_bytes;
        int32_t yr[RIN];        // grid rows loaded (wrapped when periodic)
        int32_t yw;             // first owned row of the wave
        int32_t xl;             // first column of this lane
        int32_t zs, ze;
        uint32_t lo;            // byte offset of the lane's first column
        uint32_t eo[VX];        // element offsets (element-wise access)
        uint32_t xr_off;        // this lane's outer-column element within a plane
        bool xr_zero;           // that element is an x ghost (zero rule)
        int32_t ox0, ox1;       // owned columns
        uint32_t so, out_bytes;
        int lane;
        TC w[27];
    };

    template <int TB_>
    struct State {
        TC q[TB_][3][RIN][VX];  // step l's z queue (rows used: K + 2(TB - l))
        TC xr[3];               // outer-column values of step 0's queued planes
        TC pf[RIN][VX];         // the prefetched input plane
        TC pfx;
    };

    static __device__ __forceinline__ bool ghost(int32_t i, int32_t n) {
        return !PER && static_cast<uint32_t>(i) >= static_cast<uint32_t>(n);
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
        static_assert(kBytes % 8 == 0, "whole 8-byte units per lane");
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

    // Input plane zz (already wrapped when periodic; any value under the zero rule).
    static __device__ __forceinline__ void load_plane(const Ctx& c, int32_t zz, TC (&v)[RIN][VX], TC& xr) {
        const bool zout = ghost(zz, c.nz);
        const TS* pbase = zout ? c.src : c.src + static_cast<int64_t>(zz) * c.plane_elems;
#pragma unroll
        for (int r = 0; r < RIN; ++r) {
            const bool out = zout || ghost(c.yr[r], c.ny);
            const TS* base = out ? c.src : pbase + c.yr[r] * c.nx;
            const __amdgpu_buffer_rsrc_t rs =
                __builtin_amdgcn_make_buffer_rsrc(const_cast<TS*>(base), 0, out ? 0 : c.row_bytes, kRsrcWord3);
            if constexpr (FAST) {
                bloadv(rs, c.lo, v[r]);
            } else {
#pragma unroll
                for (int e = 0; e < VX; ++e) v[r][e] = bload1(rs, c.eo[e]);
            }
        }
        const __amdgpu_buffer_rsrc_t rp =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<TS*>(pbase), 0, zout ? 0 : c.plane_bytes, kRsrcWord3);
        xr = bload1(rp, c.xr_off);
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

    // Step L on its queue (slot (J+1+s) % 3 holds plane zc - 1 + s): the
    // RO = K + 2(TB-1-L) output rows of plane zc; output row o reads queue
    // rows o .. o+2.
    template <int L, int J>
    static __device__ __forceinline__ void compute(const Ctx& c, const State<TB>& st,
                                                   TC (&out)[K + 2 * (TB - 1 - L)][VX]) {
        constexpr int RL = K + 2 * (TB - L);  // rows of this step's queue
        constexpr int RO = RL - 2;
        TC lft[3][RL], rgt[3][RL];
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int sl = (J + 1 + s) % 3;
            if constexpr (L == 0) {
                const TC xg = c.xr_zero ? TC(0) : st.xr[sl];
#pragma unroll
                for (int r = 0; r < RL; ++r) {
                    lft[s][r] = from_lower(st.q[0][sl][r][VX - 1], lane_value(xg, r));
                    rgt[s][r] = from_upper(st.q[0][sl][r][0], lane_value(xg, 32 + r));
                }
            } else {
#pragma unroll
                for (int r = 0; r < RL; ++r) {
                    lft[s][r] = from_lower_z(st.q[L][sl][r][VX - 1]);
                    rgt[s][r] = from_upper_z(st.q[L][sl][r][0]);
                }
            }
        }
#pragma unroll
        for (int o = 0; o < RO; ++o) {
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                TC acc = c.w[0] * st.q[L][(J + 2) % 3][o + 1][e];
                int p = 1;
#pragma unroll
                for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
                    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                        for (int dx = -1; dx <= 1; ++dx) {
                            if (dz == 0 && dy == 0 && dx == 0) continue;
                            const int s = dz + 1, r = o + 1 + dy, x = e + dx;
                            const int sl = (J + 1 + s) % 3;
                            const TC v = x < 0 ? lft[s][r]
                                               : (x >= VX ? rgt[s][r] : st.q[L][sl][r][x < 0 ? 0 : (x >= VX ? 0 : x)]);
                            acc = fma_c(c.w[p], v, acc);
                            ++p;
                        }
                out[o][e] = acc;
            }
        }
    }

    // Zero rule: the ghost cells of an intermediate step stay 0 (plane, rows,
    // and columns when the tile is not moved inward); bfloat16 rounds.
    template <int L>
    static __device__ __forceinline__ void finish(const Ctx& c, int32_t zc, TC (&out)[K + 2 * (TB - 1 - L)][VX]) {
        constexpr int RO = K + 2 * (TB - 1 - L);
        const bool zg = ghost(zc, c.nz);
#pragma unroll
        for (int o = 0; o < RO; ++o) {
            const bool rg = zg || ghost(c.yw - (TB - 1 - L) + o, c.ny);
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                const bool g = rg || (!FAST && ghost(c.xl + e, c.nx));
                out[o][e] = g ? TC(0) : S::round(out[o][e]);
            }
        }
    }

    static __device__ __forceinline__ void store_plane(const Ctx& c, int32_t z, const TC (&out)[K][VX]) {
        const bool zok = static_cast<uint32_t>(z - c.zs) < static_cast<uint32_t>(c.ze - c.zs);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int32_t y = c.yw + k;
            const bool ok = zok && static_cast<uint32_t>(y) < static_cast<uint32_t>(c.ny);
            TS* base = ok ? c.dst + static_cast<int64_t>(z) * c.plane_elems + y * c.nx + c.ox0 : c.dst;
            const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(base, 0, ok ? c.out_bytes : 0, kRsrcWord3);
            if constexpr (FAST) {
                bstorev(r, c.so, out[k]);
            } else {
#pragma unroll
                for (int e = 0; e < VX; ++e) bstore1(r, c.so + e * static_cast<uint32_t>(sizeof(TS)), out[k][e]);
            }
        }
    }

    static __device__ __forceinline__ int32_t wz(const Ctx& c, int32_t z) { return PER ? wrap_idx(z, c.nz) : z; }

    // Step L of the iteration that took input plane zin into slot J: plane
    // zin - (L+1); its output enters step L+1's queue at slot J.
    template <int L, int J>
    static __device__ __forceinline__ void level(const Ctx& c, int32_t zin, State<TB>& st) {
        constexpr int RO = K + 2 * (TB - 1 - L);
        TC out[RO][VX];
        compute<L, J>(c, st, out);
        const int32_t zc = zin - (L + 1);
        if constexpr (L + 1 == TB) {
            store_plane(c, zc, out);
        } else {
            finish<L>(c, zc, out);
#pragma unroll
            for (int o = 0; o < RO; ++o)
#pragma unroll
                for (int e = 0; e < VX; ++e) st.q[L + 1][J][o][e] = out[o][e];
            level<L + 1, J>(c, zin, st);
        }
    }

    template <int J>
    static __device__ __forceinline__ void step(const Ctx& c, int32_t zin, int32_t zlast, State<TB>& st) {
#pragma unroll
        for (int r = 0; r < RIN; ++r)
#pragma unroll
            for (int e = 0; e < VX; ++e) st.q[0][J][r][e] = st.pf[r][e];
        st.xr[J] = st.pfx;
        load_plane(c, wz(c, zin + 1 <= zlast ? zin + 1 : zlast), st.pf, st.pfx);
        level<0, J>(c, zin, st);
    }

    static __device__ __forceinline__ void run(const Box3DArgs& a) {
        Ctx c;
        c.lane = threadIdx.x & 63;
        const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
        const uint32_t tiles = static_cast<uint32_t>(a.tiles_x) * a.tiles_y * a.chunks_z;
        const uint32_t item = static_cast<uint32_t>(xcd_remap(blockIdx.x, gridDim.x));
        if (item >= tiles) return;
        const uint32_t txy = item / static_cast<uint32_t>(a.tiles_x);
        const int32_t tx = static_cast<int32_t>(item - txy * a.tiles_x);
        const int32_t ty = static_cast<int32_t>(txy % static_cast<uint32_t>(a.tiles_y));
        const int32_t cz = static_cast<int32_t>(txy / static_cast<uint32_t>(a.tiles_y));
        c.src = static_cast<const TS*>(a.src);
        c.dst = static_cast<TS*>(a.dst);
        c.nz = static_cast<int32_t>(a.nz);
        c.ny = static_cast<int32_t>(a.ny);
        c.nx = static_cast<int32_t>(a.nx);
        c.plane_elems = a.ny * a.nx;
        c.row_bytes = static_cast<uint32_t>(c.nx) * sizeof(TS);
        c.plane_bytes = static_cast<uint32_t>(c.plane_elems) * sizeof(TS);
        constexpr int32_t OUTW = W - 2 * HX;
        c.ox0 = tx * OUTW;
        c.ox1 = c.ox0 + OUTW < c.nx ? c.ox0 + OUTW : c.nx;
        int32_t X0 = c.ox0 - HX;
        if (!PER && FAST) X0 = X0 < 0 ? 0 : (X0 + W > c.nx ? c.nx - W : X0);
        c.xl = X0 + c.lane * VX;
        c.yw = ty * H + wave * K;
#pragma unroll
        for (int r = 0; r < RIN; ++r) c.yr[r] = PER ? wrap_idx(c.yw - TB + r, c.ny) : c.yw - TB + r;
        c.lo = static_cast<uint32_t>(PER ? wrap_idx(c.xl, c.nx) : c.xl) * sizeof(TS);
#pragma unroll
        for (int e = 0; e < VX; ++e)
            c.eo[e] = static_cast<uint32_t>(PER ? wrap_idx(c.xl + e, c.nx) : c.xl + e) * sizeof(TS);
        {
            const bool right = c.lane >= 32;
            const int r = right ? c.lane - 32 : c.lane;
            const int32_t rr = r < RIN ? r : 0;
            const int32_t xx = right ? X0 + W : X0 - 1;
            const int32_t y = c.yw - TB + rr;
            const int32_t ry = PER ? wrap_idx(y, c.ny) : y;
            const int32_t rx = PER ? wrap_idx(xx, c.nx) : xx;
            // a ghost row gives an offset outside the plane (loads 0); a ghost
            // column would read the neighbouring row and is zeroed on use
            c.xr_off = static_cast<uint32_t>(ry * c.nx + rx) * sizeof(TS);
            c.xr_zero = ghost(xx, c.nx);
        }
        c.so = static_cast<uint32_t>(c.xl - c.ox0) * sizeof(TS);
        c.out_bytes = static_cast<uint32_t>(c.ox1 - c.ox0) * sizeof(TS);
        c.zs = cz * a.chunk_z;
        c.ze = c.zs + a.chunk_z < c.nz ? c.zs + a.chunk_z : c.nz;
#pragma unroll
        for (int p = 0; p < 27; ++p) c.w[p] = static_cast<TC>(a.w[p]);

        // stream planes zs-TB .. ze-1+TB; the last step outputs plane zin-TB
        const int32_t zfirst = c.zs - TB, zlast = c.ze - 1 + TB;
        State<TB> st;
#pragma unroll
        for (int l = 0; l < TB; ++l)
#pragma unroll
            for (int s = 0; s < 3; ++s)
#pragma unroll
                for (int r = 0; r < RIN; ++r)
#pragma unroll
                    for (int e = 0; e < VX; ++e) st.q[l][s][r][e] = TC(0);
#pragma unroll
        for (int s = 0; s < 3; ++s) st.xr[s] = TC(0);
        load_plane(c, wz(c, zfirst), st.pf, st.pfx);
        int32_t zin = zfirst;
        for (; zin + 2 <= zlast; zin += 3) {
            step<0>(c, zin, zlast, st);
            step<1>(c, zin + 1, zlast, st);
            step<2>(c, zin + 2, zlast, st);
        }
        if (zin <= zlast) step<0>(c, zin, zlast, st);
        if (zin + 1 <= zlast) step<1>(c, zin + 1, zlast, st);
    }
};

template <typename TS, int VX, int K, int NW, int TB, bool PER, bool FAST>
__global__ __launch_bounds__(64 * NW) void box3d_kernel(const Box3DArgs a) {
    Kern<TS, VX, K, NW, TB, PER, FAST>::run(a);
}

template <typename TS, int VX, int K, int NW, int TB>
hipError_t launch_t(bool per, bool fast, const Box3DArgs& a, hipStream_t s) {
    const int64_t tiles = static_cast<int64_t>(a.tiles_x) * a.tiles_y * a.chunks_z;
    const dim3 grid(static_cast<unsigned>(tiles)), block(64 * NW);
    if (per) {
        if (fast) hipLaunchKernelGGL((box3d_kernel<TS, VX, K, NW, TB, true, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((box3d_kernel<TS, VX, K, NW, TB, true, false>), grid, block, 0, s, a);
    } else {
        if (fast) hipLaunchKernelGGL((box3d_kernel<TS, VX, K, NW, TB, false, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((box3d_kernel<TS, VX, K, NW, TB, false, false>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace b3d

Box3DShape box3d_shape(int dtype, int tb) {
    const int vx = dtype == kF64 ? 2 : 4;
    const int k = tb == 1 ? 4 : 2, nw = tb == 1 ? 4 : 8;
    const int hx = ((tb - 1) + vx - 1) / vx * vx;
    return Box3DShape{vx, 64 * vx, k * nw, 64 * vx - 2 * hx, 64 * nw};
}

hipError_t launch_box3d(int dtype, bool periodic, bool fast, const Box3DArgs& a, hipStream_t s) {
    if (static_cast<int64_t>(a.tiles_x) * a.tiles_y * a.chunks_z <= 0) return hipSuccess;
    if (a.tb == 1) {
        switch (dtype) {
            case kF64: return b3d::launch_t<double, 2, 4, 4, 1>(periodic, fast, a, s);
            case kF32: return b3d::launch_t<float, 4, 4, 4, 1>(periodic, fast, a, s);
            case kBF16: return b3d::launch_t<bf16s, 4, 4, 4, 1>(periodic, fast, a, s);
            default: return hipErrorInvalidValue;
        }
    }
    if (a.tb == 2) {
        switch (dtype) {
            case kF64: return b3d::launch_t<double, 2, 2, 8, 2>(periodic, fast, a, s);
            case kF32: return b3d::launch_t<float, 4, 2, 8, 2>(periodic, fast, a, s);
            case kBF16: return b3d::launch_t<bf16s, 4, 2, 8, 2>(periodic, fast, a, s);
            default: return hipErrorInvalidValue;
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace st
