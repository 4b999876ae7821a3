// varcoef_stream.hip -- the variable-coefficient heat step and its adjoint as
// z-streaming kernels (one step per pass), laid out like the constant-weight
// 3D sweep: a work-group owns an xy tile of 64*VX columns x (K rows x NW
// waves) and walks a chunk of planes; lane L of wave w holds columns
// X0 + L*VX .. +VX-1 of rows Y0 + w*K .. +K-1.  Each field (u and k; u, k
// and lambda for the adjoint) keeps planes z-1, z, z+1 in registers; the rows
// just above and below the wave's rows come from the L2 (loaded once per
// plane, one plane ahead), x neighbours from the neighbouring lane by DPP,
// and the columns just outside the tile through readlane into DPP's old
// operand.
//
// The ghost layer is produced by the loads themselves, so no face needs a
// test.  The operator (the faces visited z-, z+, y-, y+, x-, x+):
//   u'[i] = u[i] + alpha * sum_f kap_f * (u[f] - u[i]),
//   kap_f = (k[i] + k[f]) / 2 inside; across the grid edge kap = k[i], u = 0.
// Fields that are 0 on the ghost layer (u in the step, lambda in the
// adjoint) are read through buffer descriptors whose range is the row (or
// plane): a row, plane or column outside the grid reads 0.  k is read with
// clamped indices: the ghost neighbour of an edge cell reads that cell's own
// k, and (k + k) / 2 = k exactly, so the interior formula gives the edge term
// bit for bit.  In the adjoint u is read clamped too, which makes the
// interior dL/dk term (u[f] - u[i]) / 2 * (lambda[i] - lambda[f]) vanish
// across the edge; the edge term -u[i] * lambda[i] is added once per ghost
// face at the end (the count of a cell's ghost faces is fixed by its
// position).
#include <utility>

#include "dev_common.h"

namespace st {
namespace vcs {

template <typename T, int VX, int K, int NW, bool ADJ>
struct Kern {
    static constexpr int W = 64 * VX;
    static constexpr int H = NW * K;
    static constexpr int F = ADJ ? 3 : 2;  // fields: 0 u, 1 k, 2 lambda
    static constexpr int32_t kRsrcWord3 = 0x00020000;  // gfx9: raw 32-bit data
    static constexpr int32_t kNT = 2;                  // non-temporal stores
    static constexpr bool clamped(int f) { return f == 1 || (ADJ && f == 0); }

    struct Ctx {
        const T* fld[F];
        T* out;
        T* grad;
        int32_t nz, ny, nx;
        int64_t plane_elems;
        uint32_t row_bytes, plane_bytes;
        int32_t X0, Y0, yw, zs, ze;
        int32_t ox0, ox1, oy0, oy1;
        uint32_t lo;                   // byte offset of this lane's columns in a row
        uint32_t xr_zero, xr_clamp;    // x-ring element: byte offset in its plane
        bool xr_xg;                    // the x-ring element lies outside the grid
        uint32_t so, out_bytes;        // store: lane offset from ox0, output row bytes
        int ngx[VX];                   // ghost x faces of this lane's columns
        int lane, wave;
        T alpha;
    };

    static __device__ __forceinline__ bool outside(int32_t i, int32_t n) {
        return static_cast<uint32_t>(i) >= static_cast<uint32_t>(n);
    }
    static __device__ __forceinline__ int32_t clampi(int32_t i, int32_t n) { return i < 0 ? 0 : (i >= n ? n - 1 : i); }

    // one row of field f in plane z (row y): empty range outside the grid for
    // the zero fields, clamped indices for the others
    static __device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const Ctx& c, int f, int32_t z, int32_t y) {
        if (clamped(f)) {
            const T* base = c.fld[f] + static_cast<int64_t>(clampi(z, c.nz)) * c.plane_elems + clampi(y, c.ny) * c.nx;
            return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), 0, c.row_bytes, kRsrcWord3);
        }
        const bool out = outside(z, c.nz) || outside(y, c.ny);
        const T* base = out ? c.fld[f] : c.fld[f] + static_cast<int64_t>(z) * c.plane_elems + y * c.nx;
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), 0, out ? 0 : c.row_bytes, kRsrcWord3);
    }
    static __device__ __forceinline__ T ring_x(const Ctx& c, int f, int32_t z) {
        if (clamped(f)) {
            const T* base = c.fld[f] + static_cast<int64_t>(clampi(z, c.nz)) * c.plane_elems;
            const auto r = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), 0, c.plane_bytes, kRsrcWord3);
            return bload1(r, c.xr_clamp);
        }
        const bool out = outside(z, c.nz);
        const T* base = out ? c.fld[f] : c.fld[f] + static_cast<int64_t>(z) * c.plane_elems;
        const auto r = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), 0, out ? 0 : c.plane_bytes, kRsrcWord3);
        return bload1(r, c.xr_zero);
    }
    static __device__ __forceinline__ T bload1(__amdgpu_buffer_rsrc_t r, uint32_t off) {
        if constexpr (sizeof(T) == 8) return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
        else return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
    }
    static __device__ __forceinline__ void bloadv(__amdgpu_buffer_rsrc_t r, uint32_t off, T (&v)[VX]) {
        constexpr int kBytes = VX * static_cast<int>(sizeof(T));
        static_assert(kBytes % 8 == 0 && kBytes <= 32, "vector rows of 8..32 bytes");
        if constexpr (kBytes % 16 == 0) {
            u32x4 raw[kBytes / 16];
#pragma unroll
            for (int i = 0; i < kBytes / 16; ++i)
                raw[i] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(r, off + 16 * i, 0, 0));
            __builtin_memcpy(v, raw, kBytes);
        } else {
            u32x2 raw = __builtin_bit_cast(u32x2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
            __builtin_memcpy(v, &raw, kBytes);
        }
    }
    static __device__ __forceinline__ void bstorev(__amdgpu_buffer_rsrc_t r, uint32_t off, const T (&v)[VX]) {
        constexpr int kBytes = VX * static_cast<int>(sizeof(T));
        if constexpr (kBytes % 16 == 0) {
            u32x4 raw[kBytes / 16];
            __builtin_memcpy(raw, v, kBytes);
#pragma unroll
            for (int i = 0; i < kBytes / 16; ++i) __builtin_amdgcn_raw_buffer_store_b128(raw[i], r, off + 16 * i, 0, kNT);
        } else {
            u32x2 raw;
            __builtin_memcpy(&raw, v, kBytes);
            __builtin_amdgcn_raw_buffer_store_b64(raw, r, off, 0, kNT);
        }
    }

    // per-plane inputs: K rows of each field, and the neighbours of those rows
    struct Plane {
        T v[F][K][VX];
    };
    struct Ring {
        T above[F][VX], below[F][VX];  // rows yw-1 and yw+K
        T xr[F];                       // x-ring element (see Ctx)
    };

    static __device__ __forceinline__ void load_plane(const Ctx& c, int32_t z, Plane& p) {
#pragma unroll
        for (int f = 0; f < F; ++f)
#pragma unroll
            for (int k = 0; k < K; ++k) bloadv(row_rsrc(c, f, z, c.yw + k), c.lo, p.v[f][k]);
    }
    static __device__ __forceinline__ void load_ring(const Ctx& c, int32_t z, Ring& r) {
#pragma unroll
        for (int f = 0; f < F; ++f) {
            bloadv(row_rsrc(c, f, z, c.yw - 1), c.lo, r.above[f]);
            bloadv(row_rsrc(c, f, z, c.yw + K), c.lo, r.below[f]);
            r.xr[f] = ring_x(c, f, z);
        }
    }

    static __device__ __forceinline__ T lane_value(T v, int src_lane) {
        if constexpr (sizeof(T) == 8) {
            const uint64_t b = __double_as_longlong(v);
            const uint32_t lo = __builtin_amdgcn_readlane(static_cast<int>(b), src_lane);
            const uint32_t hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), src_lane);
            return __longlong_as_double((static_cast<uint64_t>(hi) << 32) | lo);
        } else {
            return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src_lane));
        }
    }

    // centre plane C with planes Pm (z-1) and Pp (z+1); output plane z
    static __device__ __forceinline__ void compute(const Ctx& c, int32_t z, const Plane& Pm, const Plane& C,
                                                   const Plane& Pp, const Ring& r) {
        const bool zok = static_cast<uint32_t>(z - c.zs) < static_cast<uint32_t>(c.ze - c.zs);
        const int ngz = (z == 0) + (z == c.nz - 1);
        T xv[F];
#pragma unroll
        for (int f = 0; f < F; ++f) xv[f] = c.xr_xg && !clamped(f) ? T(0) : r.xr[f];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            // x neighbours of the lane's first and last columns
            T lft[F], rgt[F];
#pragma unroll
            for (int f = 0; f < F; ++f) {
                lft[f] = from_lower(C.v[f][k][VX - 1], lane_value(xv[f], k));
                rgt[f] = from_upper(C.v[f][k][0], lane_value(xv[f], 32 + k));
            }
            T o[VX], g[VX];
            const int32_t y = c.yw + k;
            const int ngzy = ngz + (y == 0) + (y == c.ny - 1);
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                T nb[6][F];  // faces z-, z+, y-, y+, x-, x+
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    nb[0][f] = Pm.v[f][k][e];
                    nb[1][f] = Pp.v[f][k][e];
                    nb[2][f] = k > 0 ? C.v[f][k > 0 ? k - 1 : 0][e] : r.above[f][e];
                    nb[3][f] = k < K - 1 ? C.v[f][k < K - 1 ? k + 1 : 0][e] : r.below[f][e];
                    nb[4][f] = e > 0 ? C.v[f][k][e > 0 ? e - 1 : 0] : lft[f];
                    nb[5][f] = e < VX - 1 ? C.v[f][k][e < VX - 1 ? e + 1 : 0] : rgt[f];
                }
                const T uc = C.v[0][k][e], kc = C.v[1][k][e];
                T acc = T(0);
                if constexpr (!ADJ) {
#pragma unroll
                    for (int fc = 0; fc < 6; ++fc) {
                        const T kap = T(0.5) * (kc + nb[fc][1]);
                        acc = fma_c(kap, nb[fc][0] - uc, acc);
                    }
                    o[e] = fma_c(c.alpha, acc, uc);
                } else {
                    const T lc = C.v[2][k][e];
                    T gacc = T(0);
#pragma unroll
                    for (int fc = 0; fc < 6; ++fc) {
                        const T kap = T(0.5) * (kc + nb[fc][1]);
                        acc = fma_c(kap, nb[fc][2] - lc, acc);
                        gacc = fma_c(T(0.5) * (nb[fc][0] - uc), lc - nb[fc][2], gacc);
                    }
                    const int ng = ngzy + c.ngx[e];
                    gacc = fma_c(-static_cast<T>(ng) * uc, lc, gacc);
                    o[e] = fma_c(c.alpha, acc, lc);
                    g[e] = gacc;
                }
            }
            const bool ok = zok && static_cast<uint32_t>(y - c.oy0) < static_cast<uint32_t>(c.oy1 - c.oy0);
            const int64_t roff = static_cast<int64_t>(z) * c.plane_elems + y * c.nx + c.ox0;
            T* ob = ok ? c.out + roff : c.out;
            bstorev(__builtin_amdgcn_make_buffer_rsrc(ob, 0, ok ? c.out_bytes : 0, kRsrcWord3), c.so, o);
            if constexpr (ADJ) {
                if (c.grad != nullptr) {
                    // dL/dk += alpha * gacc (read-modify-write of this cell)
                    T* gb = ok ? c.grad + roff : c.grad;
                    const auto gr = __builtin_amdgcn_make_buffer_rsrc(gb, 0, ok ? c.out_bytes : 0, kRsrcWord3);
                    T old[VX];
                    bloadv(gr, c.so, old);
#pragma unroll
                    for (int e = 0; e < VX; ++e) g[e] = fma_c(c.alpha, g[e], old[e]);
                    bstorev(gr, c.so, g);
                }
            }
        }
    }

    struct State {
        Plane q[3];
        Ring r[2];
    };

    // iteration it: output plane z = zs + it; slots (J+2)%3, J%3, (J+1)%3 hold
    // planes z-1, z, z+1; ring buffer J%2 holds plane z's neighbours
    template <int J>
    static __device__ __forceinline__ void step(const Ctx& c, int32_t it, State& s) {
        const int32_t z = c.zs + it;
        compute(c, z, s.q[(J + 2) % 3], s.q[J % 3], s.q[(J + 1) % 3], s.r[J % 2]);
        // refill: plane z+2 into the slot of z-1, the next plane's neighbours
        load_plane(c, z + 2, s.q[(J + 2) % 3]);
        load_ring(c, z + 1, s.r[(J + 1) % 2]);
    }
    template <int... J>
    static __device__ __forceinline__ void group(const Ctx& c, int32_t base, State& s, std::integer_sequence<int, J...>) {
        (step<J>(c, base + J, s), ...);
    }
    template <int... J>
    static __device__ __forceinline__ void tail(const Ctx& c, int32_t base, int32_t nit, State& s,
                                                std::integer_sequence<int, J...>) {
        ((base + J < nit ? step<J>(c, base + J, s) : void()), ...);
    }

    static __device__ void run(const VarcoefArgs& a) {
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
        c.fld[0] = static_cast<const T*>(a.u);
        c.fld[1] = static_cast<const T*>(a.k);
        if constexpr (ADJ) c.fld[2] = static_cast<const T*>(a.lam);
        c.out = static_cast<T*>(a.out);
        c.grad = static_cast<T*>(a.grad);
        c.nz = static_cast<int32_t>(a.nz);
        c.ny = static_cast<int32_t>(a.ny);
        c.nx = static_cast<int32_t>(a.nx);
        c.plane_elems = a.ny * a.nx;
        c.row_bytes = static_cast<uint32_t>(c.nx) * sizeof(T);
        c.plane_bytes = static_cast<uint32_t>(c.plane_elems) * sizeof(T);
        c.alpha = static_cast<T>(a.alpha);
        // the register tile never overhangs the grid (the last tile in x and y
        // is moved back to end at the grid's edge); each cell is still owned,
        // and stored, by exactly one tile (the adjoint's dL/dk update is a
        // read-modify-write)
        c.ox0 = tx * W;
        c.oy0 = ty * H;
        c.ox1 = c.ox0 + W < c.nx ? c.ox0 + W : c.nx;
        c.oy1 = c.oy0 + H < c.ny ? c.oy0 + H : c.ny;
        c.X0 = c.ox0 + W > c.nx ? c.nx - W : c.ox0;
        c.Y0 = c.oy0 + H > c.ny ? c.ny - H : c.oy0;
        const int32_t xl = c.X0 + c.lane * VX;
        c.yw = c.Y0 + c.wave * K;
        c.lo = static_cast<uint32_t>(xl) * sizeof(T);
        c.so = static_cast<uint32_t>(xl - c.ox0) * sizeof(T);
        c.out_bytes = static_cast<uint32_t>(c.ox1 - c.ox0) * sizeof(T);
#pragma unroll
        for (int e = 0; e < VX; ++e) c.ngx[e] = (xl + e == 0) + (xl + e == c.nx - 1);
        {
            // lanes 0..K-1 fetch the column left of the tile for row k = lane,
            // lanes 32..32+K-1 the column right of it
            const bool right = c.lane >= 32;
            const int slot = right ? c.lane - 32 : c.lane;
            const int32_t ry = c.yw + (slot < K ? slot : 0);
            const int32_t rx = right ? c.X0 + W : c.X0 - 1;
            c.xr_xg = outside(rx, c.nx);
            c.xr_zero = static_cast<uint32_t>(ry * c.nx + rx) * sizeof(T);
            c.xr_clamp = static_cast<uint32_t>(ry * c.nx + clampi(rx, c.nx)) * sizeof(T);
        }
        c.zs = cz * a.chunk_z;
        c.ze = c.zs + a.chunk_z < c.nz ? c.zs + a.chunk_z : c.nz;
        const int32_t nit = c.ze - c.zs;

        State s;
        load_plane(c, c.zs - 1, s.q[2]);
        load_plane(c, c.zs, s.q[0]);
        load_plane(c, c.zs + 1, s.q[1]);
        load_ring(c, c.zs, s.r[0]);
        int32_t base = 0;
        for (; base + 6 <= nit; base += 6) group(c, base, s, std::make_integer_sequence<int, 6>{});
        tail(c, base, nit, s, std::make_integer_sequence<int, 6>{});
    }
};

template <typename T, int VX, int K, int NW, bool ADJ>
__global__ __launch_bounds__(64 * NW) void varcoef_stream_kernel(const VarcoefArgs a) {
    Kern<T, VX, K, NW, ADJ>::run(a);
}

}  // namespace vcs

// Streaming configuration per precision: (columns per lane, rows per wave, waves)
template <typename T> struct VcsCfg;
template <> struct VcsCfg<float> { static constexpr int VX = 4, KF = 4, KA = 2, NW = 4; };
template <> struct VcsCfg<double> { static constexpr int VX = 2, KF = 4, KA = 2, NW = 4; };

template <typename T>
static void vcs_shape(bool adjoint, int& w, int& h, int& block) {
    w = 64 * VcsCfg<T>::VX;
    h = (adjoint ? VcsCfg<T>::KA : VcsCfg<T>::KF) * VcsCfg<T>::NW;
    block = 64 * VcsCfg<T>::NW;
}

void varcoef_stream_shape(int dtype, bool adjoint, int& w, int& h, int& block) {
    if (dtype == kF64) vcs_shape<double>(adjoint, w, h, block);
    else vcs_shape<float>(adjoint, w, h, block);
}

template <typename T>
static hipError_t vcs_launch(bool adjoint, const VarcoefArgs& a, hipStream_t s) {
    using C = VcsCfg<T>;
    const int64_t wgs = static_cast<int64_t>(a.tiles_x) * a.tiles_y * a.chunks_z;
    if (wgs <= 0) return hipSuccess;
    if (wgs >= (int64_t(1) << 31)) return hipErrorInvalidValue;
    const dim3 grid(static_cast<unsigned>(wgs)), block(64 * C::NW);
    if (adjoint) hipLaunchKernelGGL((vcs::varcoef_stream_kernel<T, C::VX, C::KA, C::NW, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((vcs::varcoef_stream_kernel<T, C::VX, C::KF, C::NW, false>), grid, block, 0, s, a);
    return hipGetLastError();
}

template <typename T>
static int vcs_occ(bool adjoint) {
    using C = VcsCfg<T>;
    int n = 0;
    hipError_t e = adjoint
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, vcs::varcoef_stream_kernel<T, C::VX, C::KA, C::NW, true>, 64 * C::NW, 0)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, vcs::varcoef_stream_kernel<T, C::VX, C::KF, C::NW, false>, 64 * C::NW, 0);
    return e == hipSuccess ? n : 0;
}

int varcoef_stream_occupancy(int dtype, bool adjoint) {
    // asked once per (precision, direction); the library drives one GPU model
    static int cache[2][2] = {{-1, -1}, {-1, -1}};
    int& v = cache[dtype == kF64 ? 1 : 0][adjoint ? 1 : 0];
    if (v < 0) v = dtype == kF64 ? vcs_occ<double>(adjoint) : vcs_occ<float>(adjoint);
    return v;
}

hipError_t launch_varcoef_stream(int dtype, bool adjoint, const VarcoefArgs& a, hipStream_t s) {
    if (dtype == kF64) return vcs_launch<double>(adjoint, a, s);
    if (dtype == kF32) return vcs_launch<float>(adjoint, a, s);
    return hipErrorInvalidValue;
}

}  // namespace st
