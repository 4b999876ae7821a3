// stream1d.hip -- 1D stars (radius R, all 2R+1 points) with T_b steps per
// pass, the whole space-time tile in registers.
//
// Paper Sec. 4.1 tiles 1D space-time into trapezoids that carry several time
// steps per load; on gfx950 one wave holds a strip of 64*VX consecutive cells
// (lane L: cells X0 + L*VX .. + VX - 1), and each step needs from the
// neighbouring lanes only their R edge cells, moved by DPP wave shifts (a
// zero enters at the wave's ends).  After t steps the cells within R*t of
// the strip's ends are stale, so a strip owns its middle 64*VX - 2H cells
// (H >= R*T_b, a multiple of VX) and neighbouring strips overlap by 2H.
//
// Zero rule, whole-vector rows (n % VX == 0, n >= 64*VX, 16-byte aligned):
// the strips at the grid's ends are moved inward to start at 0 / end at n,
// where the zero entering through DPP is exactly the ghost cell; no masks.
// Otherwise (short or unaligned grids) cells outside [0, n) are loaded as 0
// (buffer range) and set back to 0 after every step.  Periodic: strips keep
// their place and every index wraps (lanes whose cells straddle the wrap
// load them one by one).
//
// Canonical point order: centre, then offsets -R..-1, +1..+R, one multiply
// then an FMA chain -- the same arithmetic as the one-step kernel, so every
// depth gives the same bits.
#include "dev_common.h"

namespace st {
namespace s1d {

template <typename TS, int R, int VX, bool PER>
struct Kern {
    using S = Storage<TS>;
    using TC = typename S::TC;
    static_assert(VX >= R, "a lane must hold at least R cells");
    static constexpr int W = 64 * VX;
    static constexpr int NP = 2 * R + 1;
    static constexpr int32_t kRsrcWord3 = 0x00020000;  // gfx9: raw 32-bit data
    static constexpr int32_t kNT = 2;                  // store cache policy: non-temporal

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
        static_assert(kBytes % 16 == 0, "whole 16-byte units per lane");
        TS vals[VX];
        u32x4 raw[kBytes / 16];
#pragma unroll
        for (int i = 0; i < kBytes / 16; ++i)
            raw[i] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(r, off + 16 * i, 0, 0));
        __builtin_memcpy(vals, raw, kBytes);
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
        u32x4 raw[kBytes / 16];
        __builtin_memcpy(raw, vals, kBytes);
#pragma unroll
        for (int i = 0; i < kBytes / 16; ++i) __builtin_amdgcn_raw_buffer_store_b128(raw[i], r, off + 16 * i, 0, kNT);
    }

    // One step on the strip.  left[j] is cell xl - R + j (lane L-1's cell
    // VX - R + j), right[j] cell xl + VX + j (lane L+1's cell j).
    static __device__ __forceinline__ void step(const TC (&w)[NP], const TC (&v)[VX], TC (&out)[VX]) {
        TC left[R], right[R];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            left[j] = from_lower_z(v[VX - R + j]);
            right[j] = from_upper_z(v[j]);
        }
#pragma unroll
        for (int e = 0; e < VX; ++e) {
            TC acc = w[0] * v[e];
            int p = 1;
#pragma unroll
            for (int dx = -R; dx <= -1; ++dx, ++p) acc = fma_c(w[p], e + dx >= 0 ? v[e + dx] : left[R + e + dx], acc);
#pragma unroll
            for (int dx = 1; dx <= R; ++dx, ++p)
                acc = fma_c(w[p], e + dx < VX ? v[e + dx] : right[e + dx - VX], acc);
            out[e] = acc;
        }
    }

    template <bool FAST>
    static __device__ __forceinline__ void body(const Stream1DArgs& a, int32_t n, int32_t xl, int32_t ofirst,
                                                int32_t olast, int tb, const TC (&w)[NP]) {
        const TS* src = static_cast<const TS*>(a.src);
        TS* dst = static_cast<TS*>(a.dst);
        const __amdgpu_buffer_rsrc_t rin =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<TS*>(src), 0, static_cast<uint32_t>(n) * sizeof(TS), kRsrcWord3);
        TC v[VX];
        if constexpr (FAST && !PER) {
            bloadv(rin, static_cast<uint32_t>(xl) * sizeof(TS), v);
        } else if constexpr (FAST) {
            if (xl >= 0 && xl + VX <= n) {
                bloadv(rin, static_cast<uint32_t>(xl) * sizeof(TS), v);
            } else {
#pragma unroll
                for (int e = 0; e < VX; ++e) v[e] = bload1(rin, static_cast<uint32_t>(wrap_idx(xl + e, n)) * sizeof(TS));
            }
        } else {
            // ghost cells (zero rule) become offsets past the range: 0
#pragma unroll
            for (int e = 0; e < VX; ++e)
                v[e] = bload1(rin, static_cast<uint32_t>(PER ? wrap_idx(xl + e, n) : xl + e) * sizeof(TS));
        }
        for (int t = 0; t < tb; ++t) {
            TC out[VX];
            step(w, v, out);
            const bool last = t + 1 == tb;
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                TC o = out[e];
                if constexpr (!FAST && !PER) o = static_cast<uint32_t>(xl + e) >= static_cast<uint32_t>(n) ? TC(0) : o;
                // bfloat16 storage rounds every step (the store rounds the last)
                v[e] = last ? o : S::round(o);
            }
        }
        // owned cells [ofirst, olast): stores outside the range are dropped
        TS* base = dst + ofirst;
        const __amdgpu_buffer_rsrc_t rout =
            __builtin_amdgcn_make_buffer_rsrc(base, 0, static_cast<uint32_t>(olast - ofirst) * sizeof(TS), kRsrcWord3);
        const uint32_t so = static_cast<uint32_t>(xl - ofirst) * sizeof(TS);
        if constexpr (FAST) {
            bstorev(rout, so, v);
        } else {
#pragma unroll
            for (int e = 0; e < VX; ++e) bstore1(rout, so + e * static_cast<uint32_t>(sizeof(TS)), v[e]);
        }
    }

    static __device__ __forceinline__ void run(const Stream1DArgs& a) {
        const int lane = threadIdx.x & 63;
        const int64_t strip = __builtin_amdgcn_readfirstlane(
            static_cast<int>(xcd_remap(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6)));
        if (strip >= a.strips) return;
        const int32_t n = static_cast<int32_t>(a.n);
        const int32_t ofirst = static_cast<int32_t>(strip) * a.out_w;
        const int32_t olast = ofirst + a.out_w < n ? ofirst + a.out_w : n;
        int32_t X0 = ofirst - a.halo;
        if (!PER && a.vec_ok) X0 = X0 < 0 ? 0 : (X0 + W > n ? n - W : X0);
        const int32_t xl = X0 + lane * VX;
        TC w[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) w[p] = static_cast<TC>(a.w[p]);
        if (a.vec_ok) body<true>(a, n, xl, ofirst, olast, a.tb, w);
        else body<false>(a, n, xl, ofirst, olast, a.tb, w);
    }
};

template <typename TS, int R, int VX, bool PER>
__global__ __launch_bounds__(256) void stream1d_kernel(const Stream1DArgs a) {
    Kern<TS, R, VX, PER>::run(a);
}

template <typename TS, int R, int VX, bool PER>
hipError_t launch_t(const Stream1DArgs& a, hipStream_t s) {
    const int64_t wgs = (a.strips + 3) / 4;
    hipLaunchKernelGGL((stream1d_kernel<TS, R, VX, PER>), dim3(static_cast<unsigned>(wgs)), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename TS, int VX>
hipError_t launch_r(int radius, bool per, const Stream1DArgs& a, hipStream_t s) {
    switch (radius * 2 + (per ? 1 : 0)) {
        case 2: return launch_t<TS, 1, VX, false>(a, s);
        case 3: return launch_t<TS, 1, VX, true>(a, s);
        case 4: return launch_t<TS, 2, VX, false>(a, s);
        case 5: return launch_t<TS, 2, VX, true>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace s1d

bool stream1d_has(int dtype, int radius) {
    return (dtype == kF64 || dtype == kF32 || dtype == kBF16) && (radius == 1 || radius == 2);
}

hipError_t launch_stream1d(int dtype, int radius, bool periodic, const Stream1DArgs& a, hipStream_t s) {
    if (a.strips <= 0) return hipSuccess;
    switch (dtype) {
        case kF64: return s1d::launch_r<double, kStream1DVX>(radius, periodic, a, s);
        case kF32: return s1d::launch_r<float, kStream1DVX>(radius, periodic, a, s);
        case kBF16: return s1d::launch_r<bf16s, kStream1DVX>(radius, periodic, a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace st
