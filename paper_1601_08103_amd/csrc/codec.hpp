// Storage codecs for the population arrays.
//
// F64 / F32 store g itself.  F16 / BF16 store h = S g / f* (S a power of two), rounded to
// nearest-even; I16 stores the same h as a signed 16-bit integer (fixed point, rounded to
// nearest-even, saturating at +-32767).  The collision is computed in FP32 on the decoded h,
// with the constants folded so that no per-population rescaling is needed in the step kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));

struct StF64 {
    using elem = double;
    using comp = double;
    static constexpr bool scaled = false;
    __device__ static comp dec(elem v) { return v; }
    __device__ static elem enc(comp v) { return v; }
    __device__ static elem enc_d(double v) { return v; }
};

struct StF32 {
    using elem = float;
    using comp = float;
    static constexpr bool scaled = false;
    __device__ static comp dec(elem v) { return v; }
    __device__ static elem enc(comp v) { return v; }
    __device__ static elem enc_d(double v) { return (float)v; }
};

struct StF16 {
    using elem = unsigned short;
    using comp = float;
    static constexpr bool scaled = true;
    __device__ static comp dec(elem v) { return (float)__builtin_bit_cast(_Float16, v); }
    // v_cvt_f16_f32 rounds with the default mode: to nearest, ties to even.
    __device__ static elem enc(comp v) { return __builtin_bit_cast(unsigned short, (_Float16)v); }
    __device__ static elem enc_d(double v) { return __builtin_bit_cast(unsigned short, (_Float16)v); }
};

struct StBF16 {
    using elem = unsigned short;
    using comp = float;
    static constexpr bool scaled = true;
    __device__ static comp dec(elem v) { return __uint_as_float(((unsigned)v) << 16); }
    // Round to nearest, ties to even, on the upper 16 bits of the FP32 pattern.  Finite
    // inputs only (the state of a stable run never holds NaN or Inf).
    __device__ static elem enc(comp v) {
        unsigned u = __float_as_uint(v);
        u += 0x7fffu + ((u >> 16) & 1u);
        return (elem)(u >> 16);
    }
    __device__ static elem enc_d(double v) { return enc((float)v); }
};

struct StI16 {
    using elem = short;
    using comp = float;
    static constexpr bool scaled = true;
    __device__ static comp dec(elem v) { return (float)v; }
    __device__ static elem enc(comp v) {
        const float r = __builtin_rintf(v);  // ties to even
        return (elem)(int)fminf(fmaxf(r, -32767.0f), 32767.0f);
    }
    __device__ static elem enc_d(double v) {
        const double r = __builtin_rint(v);
        return (elem)(int)fmin(fmax(r, -32767.0), 32767.0);
    }
};

// E3M12: 1 sign bit, 3 exponent bits, 12 mantissa bits.  value = (-1)^s (1 + m/4096) 2^(e-7)
// for e >= 1 (binades [2^-6, 2)), (-1)^s m 2^-18 for e = 0 (subnormals, same spacing as the
// lowest binade).  Encoding rounds to nearest even and saturates at 2 - 2^-12 (the largest
// finite value); S is chosen so the initial |h| stays below 1, leaving one binade of headroom.
struct StE3M12 {
    using elem = unsigned short;
    using comp = float;
    static constexpr bool scaled = true;
    // e and m go to the FP32 exponent / mantissa fields (exponent field e, mantissa m << 11);
    // scaling by 2^120 then gives 2^(e-7) (1 + m/4096) for e >= 1, and for e = 0 the FP32
    // denormal m 2^-138 becomes m 2^-18.  Exact; needs FP32 denormals enabled (the kernels'
    // default float mode).
    __device__ static comp dec(elem v) {
        const unsigned x = ((unsigned)v) << 16;
        const unsigned bits = ((x >> 5) & 0x03fff800u) | (x & 0x80000000u);
        return __uint_as_float(bits) * 0x1p120f;
    }
    __device__ static elem enc(comp v) {
        const unsigned bits = __float_as_uint(v);
        const unsigned b = bits & 0x7fffffffu;
        // |v| >= 2^-6: round the 23-bit mantissa to 12 bits, ties to even, exponent rebased by
        // 120 (done before the shift), saturating at the largest code
        const unsigned rn = min((b - (120u << 23) + 0x3ffu + ((b >> 11) & 1u)) >> 11, 0x7fffu);
        // subnormal range, a multiple of 2^-18: FP32 numbers in [32, 64) are spaced 2^-18 apart,
        // so |v| + 32 rounds |v| to it (ties to even) and its low bits are the code
        const unsigned rs = __float_as_uint(__builtin_fabsf(v) + 32.0f) - 0x42000000u;
        return (elem)((b >= (121u << 23) ? rn : rs) | ((bits >> 16) & 0x8000u));
    }
    __device__ static elem enc_d(double v) { return enc((float)v); }
};

// Four consecutive elements starting at a 4-element-aligned index, decoded to the compute type.
// Vector loads/stores; NT selects the non-temporal (streaming) cache policy.
template <typename V>
__device__ __forceinline__ V vload(const V *p, bool nt) {
    return nt ? __builtin_nontemporal_load(p) : *p;
}
template <typename V>
__device__ __forceinline__ void vstore(V *p, V v, bool nt) {
    if (nt)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

template <class ST>
__device__ inline void load4(const typename ST::elem *p, typename ST::comp (&v)[4], bool nt = false);

template <>
__device__ inline void load4<StF64>(const double *p, double (&v)[4], bool nt) {
    f64x2 a = vload(reinterpret_cast<const f64x2 *>(p), nt);
    f64x2 b = vload(reinterpret_cast<const f64x2 *>(p + 2), nt);
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
template <>
__device__ inline void load4<StF32>(const float *p, float (&v)[4], bool nt) {
    f32x4 a = vload(reinterpret_cast<const f32x4 *>(p), nt);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}
template <>
__device__ inline void load4<StF16>(const unsigned short *p, float (&v)[4], bool nt) {
    u16x4 a = vload(reinterpret_cast<const u16x4 *>(p), nt);
    v[0] = StF16::dec(a.x); v[1] = StF16::dec(a.y); v[2] = StF16::dec(a.z); v[3] = StF16::dec(a.w);
}
template <>
__device__ inline void load4<StBF16>(const unsigned short *p, float (&v)[4], bool nt) {
    u16x4 a = vload(reinterpret_cast<const u16x4 *>(p), nt);
    v[0] = StBF16::dec(a.x); v[1] = StBF16::dec(a.y); v[2] = StBF16::dec(a.z); v[3] = StBF16::dec(a.w);
}

template <>
__device__ inline void load4<StE3M12>(const unsigned short *p, float (&v)[4], bool nt) {
    u16x4 a = vload(reinterpret_cast<const u16x4 *>(p), nt);
    v[0] = StE3M12::dec(a.x); v[1] = StE3M12::dec(a.y); v[2] = StE3M12::dec(a.z); v[3] = StE3M12::dec(a.w);
}

template <>
__device__ inline void load4<StI16>(const short *p, float (&v)[4], bool nt) {
    s16x4 a = vload(reinterpret_cast<const s16x4 *>(p), nt);
    v[0] = StI16::dec(a.x); v[1] = StI16::dec(a.y); v[2] = StI16::dec(a.z); v[3] = StI16::dec(a.w);
}

template <class ST>
__device__ inline void store4(typename ST::elem *p, const typename ST::comp (&v)[4], bool nt = false);

template <>
__device__ inline void store4<StF64>(double *p, const double (&v)[4], bool nt) {
    f64x2 a = {v[0], v[1]}, b = {v[2], v[3]};
    vstore(reinterpret_cast<f64x2 *>(p), a, nt);
    vstore(reinterpret_cast<f64x2 *>(p + 2), b, nt);
}
template <>
__device__ inline void store4<StF32>(float *p, const float (&v)[4], bool nt) {
    f32x4 a = {v[0], v[1], v[2], v[3]};
    vstore(reinterpret_cast<f32x4 *>(p), a, nt);
}
template <>
__device__ inline void store4<StF16>(unsigned short *p, const float (&v)[4], bool nt) {
    u16x4 a = {StF16::enc(v[0]), StF16::enc(v[1]), StF16::enc(v[2]), StF16::enc(v[3])};
    vstore(reinterpret_cast<u16x4 *>(p), a, nt);
}
template <>
__device__ inline void store4<StBF16>(unsigned short *p, const float (&v)[4], bool nt) {
    u16x4 a = {StBF16::enc(v[0]), StBF16::enc(v[1]), StBF16::enc(v[2]), StBF16::enc(v[3])};
    vstore(reinterpret_cast<u16x4 *>(p), a, nt);
}

template <>
__device__ inline void store4<StE3M12>(unsigned short *p, const float (&v)[4], bool nt) {
    u16x4 a = {StE3M12::enc(v[0]), StE3M12::enc(v[1]), StE3M12::enc(v[2]), StE3M12::enc(v[3])};
    vstore(reinterpret_cast<u16x4 *>(p), a, nt);
}

template <>
__device__ inline void store4<StI16>(short *p, const float (&v)[4], bool nt) {
    s16x4 a = {StI16::enc(v[0]), StI16::enc(v[1]), StI16::enc(v[2]), StI16::enc(v[3])};
    vstore(reinterpret_cast<s16x4 *>(p), a, nt);
}

// Two consecutive elements starting at an even index: one 16-, 8- or 4-byte access.
template <class ST>
__device__ inline void load2(const typename ST::elem *p, typename ST::comp (&v)[2], bool nt = false) {
    using E = typename ST::elem;
    typedef E e2 __attribute__((ext_vector_type(2)));
    const e2 a = vload(reinterpret_cast<const e2 *>(p), nt);
    v[0] = ST::dec(a.x);
    v[1] = ST::dec(a.y);
}
template <class ST>
__device__ inline void store2(typename ST::elem *p, const typename ST::comp (&v)[2], bool nt = false) {
    using E = typename ST::elem;
    typedef E e2 __attribute__((ext_vector_type(2)));
    const e2 a = {ST::enc(v[0]), ST::enc(v[1])};
    vstore(reinterpret_cast<e2 *>(p), a, nt);
}

}  // namespace lbm
