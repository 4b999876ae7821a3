// dev_common.h -- device helpers shared by the stencil kernels (gfx950).
//
// Storage/compute conversion, wavefront neighbour exchange with DPP, and the
// XCD-aware work-group remap.  Every kernel evaluates a point list in the
// same canonical order with the same multiply / fused-multiply-add chain, so
// that all kernels, tilings and fused depths of one plan agree bit for bit:
//   acc = w[0] * centre;  acc = fma(w[p], v[p], acc) for p = 1 .. npoints-1
// where a neighbour on the zero ghost layer contributes v[p] = 0.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace st {

// ---------------------------------------------------------------------------
// storage <-> compute
// ---------------------------------------------------------------------------
struct bf16s {
    uint16_t bits;
};

template <typename TS> struct Storage;
template <> struct Storage<double> {
    using TC = double;
    static __device__ __forceinline__ double widen(double v) { return v; }
    static __device__ __forceinline__ double narrow(double v) { return v; }
    static __device__ __forceinline__ double round(double v) { return v; }
};
template <> struct Storage<float> {
    using TC = float;
    static __device__ __forceinline__ float widen(float v) { return v; }
    static __device__ __forceinline__ float narrow(float v) { return v; }
    static __device__ __forceinline__ float round(float v) { return v; }
};
// bfloat16 storage, FP32 compute: widen exactly, narrow with round to
// nearest even through gfx950's v_cvt_pk_bf16_f32 (NaN stays a quiet NaN).
__device__ __forceinline__ float bf16_to_f32(uint16_t b) {
    return __uint_as_float(static_cast<uint32_t>(b) << 16);
}
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    return __builtin_bit_cast(uint16_t, static_cast<__bf16>(f));
}
template <> struct Storage<bf16s> {
    using TC = float;
    static __device__ __forceinline__ float widen(bf16s v) { return bf16_to_f32(v.bits); }
    static __device__ __forceinline__ bf16s narrow(float v) { return bf16s{f32_to_bf16(v)}; }
    static __device__ __forceinline__ float round(float v) { return bf16_to_f32(f32_to_bf16(v)); }
};

// Grid memory is always addressed through global (address space 1)
// pointers, so loads and stores are global_* instructions (not flat ones,
// which would also tie up the LDS counter).
#define ST_GLOBAL __attribute__((address_space(1)))

template <typename T>
__device__ __forceinline__ const ST_GLOBAL T* gptr(const void* p) {
    return (const ST_GLOBAL T*)(p);
}
template <typename T>
__device__ __forceinline__ ST_GLOBAL T* gptr_mut(void* p) {
    return (ST_GLOBAL T*)(p);
}

// Wave-uniform copies (SGPRs) of values read through a pointer.
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<int32_t>(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<int32_t>(v >> 32));
    return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}
__device__ __forceinline__ double uni(double v) { return __longlong_as_double(uni(static_cast<int64_t>(__double_as_longlong(v)))); }
__device__ __forceinline__ const void* uni(const void* p) {
    return reinterpret_cast<const void*>(uni(reinterpret_cast<int64_t>(p)));
}
__device__ __forceinline__ void* uni(void* p) { return reinterpret_cast<void*>(uni(reinterpret_cast<int64_t>(p))); }

// Scalar element access with the storage conversion.
template <typename TS>
__device__ __forceinline__ typename Storage<TS>::TC ld1(const ST_GLOBAL TS* p) {
    if constexpr (sizeof(TS) == 2) {
        return bf16_to_f32(*reinterpret_cast<const ST_GLOBAL uint16_t*>(p));
    } else {
        return Storage<TS>::widen(*p);
    }
}
template <typename TS>
__device__ __forceinline__ void st1(ST_GLOBAL TS* p, typename Storage<TS>::TC v) {
    TS s = Storage<TS>::narrow(v);
    if constexpr (sizeof(TS) == 8) {
        __builtin_nontemporal_store(__builtin_bit_cast(uint64_t, s), reinterpret_cast<ST_GLOBAL uint64_t*>(p));
    } else if constexpr (sizeof(TS) == 4) {
        __builtin_nontemporal_store(__builtin_bit_cast(uint32_t, s), reinterpret_cast<ST_GLOBAL uint32_t*>(p));
    } else {
        __builtin_nontemporal_store(__builtin_bit_cast(uint16_t, s), reinterpret_cast<ST_GLOBAL uint16_t*>(p));
    }
}

// Whole-vector access to VX consecutive elements (VX*sizeof(TS) a multiple of
// 8 bytes, the address aligned to that size, at most 16 bytes per access).
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <typename TS, int VX>
__device__ __forceinline__ void ldv(const ST_GLOBAL TS* p, typename Storage<TS>::TC (&out)[VX]) {
    constexpr int kBytes = VX * static_cast<int>(sizeof(TS));
    static_assert(kBytes % 8 == 0, "vector access needs whole 8-byte units");
    TS vals[VX];
    if constexpr (kBytes % 16 == 0) {
        constexpr int kN = kBytes / 16;
        u32x4 raw[kN];
        const ST_GLOBAL u32x4* q = reinterpret_cast<const ST_GLOBAL u32x4*>(p);
#pragma unroll
        for (int c = 0; c < kN; ++c) raw[c] = q[c];
        __builtin_memcpy(vals, raw, kBytes);
    } else {
        constexpr int kN = kBytes / 8;
        u32x2 raw[kN];
        const ST_GLOBAL u32x2* q = reinterpret_cast<const ST_GLOBAL u32x2*>(p);
#pragma unroll
        for (int c = 0; c < kN; ++c) raw[c] = q[c];
        __builtin_memcpy(vals, raw, kBytes);
    }
#pragma unroll
    for (int e = 0; e < VX; ++e) out[e] = Storage<TS>::widen(vals[e]);
}

template <typename TS, int VX>
__device__ __forceinline__ void stv(ST_GLOBAL TS* p, const typename Storage<TS>::TC (&in)[VX]) {
    constexpr int kBytes = VX * static_cast<int>(sizeof(TS));
    static_assert(kBytes % 8 == 0, "vector access needs whole 8-byte units");
    TS vals[VX];
#pragma unroll
    for (int e = 0; e < VX; ++e) vals[e] = Storage<TS>::narrow(in[e]);
    if constexpr (kBytes % 16 == 0) {
        constexpr int kN = kBytes / 16;
        u32x4 raw[kN];
        __builtin_memcpy(raw, vals, kBytes);
        ST_GLOBAL u32x4* q = reinterpret_cast<ST_GLOBAL u32x4*>(p);
#pragma unroll
        for (int c = 0; c < kN; ++c) __builtin_nontemporal_store(raw[c], q + c);
    } else {
        constexpr int kN = kBytes / 8;
        u32x2 raw[kN];
        __builtin_memcpy(raw, vals, kBytes);
        ST_GLOBAL u32x2* q = reinterpret_cast<ST_GLOBAL u32x2*>(p);
#pragma unroll
        for (int c = 0; c < kN; ++c) __builtin_nontemporal_store(raw[c], q + c);
    }
}

__device__ __forceinline__ double fma_c(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_c(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// ---------------------------------------------------------------------------
// wavefront shifts (GFX9 DPP wave_shl:1 / wave_shr:1)
// ---------------------------------------------------------------------------
// from_lower(v, old): lane i receives v from lane i-1; lane 0 receives `old`.
// from_upper(v, old): lane i receives v from lane i+1; lane 63 receives `old`.
constexpr int kDppWaveShl1 = 0x130;
constexpr int kDppWaveShr1 = 0x138;

__device__ __forceinline__ int dpp_from_lower_i(int v, int old) {
    return __builtin_amdgcn_update_dpp(old, v, kDppWaveShr1, 0xF, 0xF, false);
}
__device__ __forceinline__ int dpp_from_upper_i(int v, int old) {
    return __builtin_amdgcn_update_dpp(old, v, kDppWaveShl1, 0xF, 0xF, false);
}
__device__ __forceinline__ float from_lower(float v, float old) {
    return __int_as_float(dpp_from_lower_i(__float_as_int(v), __float_as_int(old)));
}
__device__ __forceinline__ float from_upper(float v, float old) {
    return __int_as_float(dpp_from_upper_i(__float_as_int(v), __float_as_int(old)));
}
// Same with 0 entering at the wave's edge (bound_ctrl): one instruction per
// dword, no initialisation of the destination.
__device__ __forceinline__ int dpp_from_lower_z(int v) { return __builtin_amdgcn_mov_dpp(v, kDppWaveShr1, 0xF, 0xF, true); }
__device__ __forceinline__ int dpp_from_upper_z(int v) { return __builtin_amdgcn_mov_dpp(v, kDppWaveShl1, 0xF, 0xF, true); }
__device__ __forceinline__ float from_lower_z(float v) { return __int_as_float(dpp_from_lower_z(__float_as_int(v))); }
__device__ __forceinline__ float from_upper_z(float v) { return __int_as_float(dpp_from_upper_z(__float_as_int(v))); }
__device__ __forceinline__ double from_lower_z(double v) {
    const uint64_t b = __double_as_longlong(v);
    const uint32_t lo = static_cast<uint32_t>(dpp_from_lower_z(static_cast<int>(b)));
    const uint32_t hi = static_cast<uint32_t>(dpp_from_lower_z(static_cast<int>(b >> 32)));
    return __longlong_as_double((static_cast<uint64_t>(hi) << 32) | lo);
}
__device__ __forceinline__ double from_upper_z(double v) {
    const uint64_t b = __double_as_longlong(v);
    const uint32_t lo = static_cast<uint32_t>(dpp_from_upper_z(static_cast<int>(b)));
    const uint32_t hi = static_cast<uint32_t>(dpp_from_upper_z(static_cast<int>(b >> 32)));
    return __longlong_as_double((static_cast<uint64_t>(hi) << 32) | lo);
}
__device__ __forceinline__ double from_lower(double v, double old) {
    const uint64_t b = __double_as_longlong(v), o = __double_as_longlong(old);
    const int lo = dpp_from_lower_i(static_cast<int>(b), static_cast<int>(o));
    const int hi = dpp_from_lower_i(static_cast<int>(b >> 32), static_cast<int>(o >> 32));
    return __longlong_as_double((static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) |
                                static_cast<uint32_t>(lo));
}
__device__ __forceinline__ double from_upper(double v, double old) {
    const uint64_t b = __double_as_longlong(v), o = __double_as_longlong(old);
    const int lo = dpp_from_upper_i(static_cast<int>(b), static_cast<int>(o));
    const int hi = dpp_from_upper_i(static_cast<int>(b >> 32), static_cast<int>(o >> 32));
    return __longlong_as_double((static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) |
                                static_cast<uint32_t>(lo));
}

// ---------------------------------------------------------------------------
// XCD-aware work-group order
// ---------------------------------------------------------------------------
// The dispatcher hands work-group b to XCD (b mod 8).  Renumbering so that each
// XCD receives one contiguous range of logical tiles keeps tiles that share
// halo cells inside one L2.  A bijection for any count.
// Sum over the 64 lanes of a wave (butterfly through ds_swizzle/bpermute;
// every lane's order of additions is fixed, so the result is reproducible).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nblocks) {
    constexpr int64_t kXcd = 8;
    const int64_t q = nblocks / kXcd, r = nblocks % kXcd;
    const int64_t x = b % kXcd, k = b / kXcd;
    return x * q + (x < r ? x : r) + k;
}

__device__ __forceinline__ int64_t wrap_idx(int64_t i, int64_t n) {
    i %= n;
    return i < 0 ? i + n : i;
}
__device__ __forceinline__ int32_t wrap_idx(int32_t i, int32_t n) {
    i %= n;
    return i < 0 ? i + n : i;
}

}  // namespace st
