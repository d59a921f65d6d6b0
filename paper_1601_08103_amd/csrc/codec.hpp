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

struct StF64 {
    using elem = double;
    using comp = double;
    static constexpr bool scaled = false;
    // raw domain of the step kernels (see StE3M12); identical to the real domain here
    static constexpr bool has_raw = false;
    static constexpr double raw_unit = 1.0;
    __device__ static comp dec_raw(elem v) { return dec(v); }
    __device__ static elem enc_raw(comp v) { return enc(v); }
    __device__ static comp dec(elem v) { return v; }
    __device__ static elem enc(comp v) { return v; }
    __device__ static elem enc_d(double v) { return v; }
};

struct StF32 {
    using elem = float;
    using comp = float;
    static constexpr bool scaled = false;
    // raw domain of the step kernels (see StE3M12); identical to the real domain here
    static constexpr bool has_raw = false;
    static constexpr double raw_unit = 1.0;
    __device__ static comp dec_raw(elem v) { return dec(v); }
    __device__ static elem enc_raw(comp v) { return enc(v); }
    __device__ static comp dec(elem v) { return v; }
    __device__ static elem enc(comp v) { return v; }
    __device__ static elem enc_d(double v) { return (float)v; }
};

struct StF16 {
    using elem = unsigned short;
    using comp = float;
    static constexpr bool scaled = true;
    // raw domain of the step kernels (see StE3M12); identical to the real domain here
    static constexpr bool has_raw = false;
    static constexpr double raw_unit = 1.0;
    __device__ static comp dec_raw(elem v) { return dec(v); }
    __device__ static elem enc_raw(comp v) { return enc(v); }
    __device__ static comp dec(elem v) { return (float)__builtin_bit_cast(_Float16, v); }
    // v_cvt_f16_f32 rounds with the default mode: to nearest, ties to even.  The input is
    // first fixed as an FP32 value: without the empty asm the compiler fuses the conversion
    // into the fma that produced v (v_fma_mixlo_f16, one rounding straight to FP16) for some
    // stores and not for others, depending on how a kernel packs them, and two kernels with
    // the same arithmetic would differ in the last FP16 bit.
    __device__ static elem enc(comp v) {
        __asm__("" : "+v"(v));
        return __builtin_bit_cast(unsigned short, (_Float16)v);
    }
    __device__ static elem enc_d(double v) { return __builtin_bit_cast(unsigned short, (_Float16)v); }
};

struct StBF16 {
    using elem = unsigned short;
    using comp = float;
    static constexpr bool scaled = true;
    // raw domain of the step kernels (see StE3M12); identical to the real domain here
    static constexpr bool has_raw = false;
    static constexpr double raw_unit = 1.0;
    __device__ static comp dec_raw(elem v) { return dec(v); }
    __device__ static elem enc_raw(comp v) { return enc(v); }
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
    // raw domain of the step kernels (see StE3M12); identical to the real domain here
    static constexpr bool has_raw = false;
    static constexpr double raw_unit = 1.0;
    __device__ static comp dec_raw(elem v) { return dec(v); }
    __device__ static elem enc_raw(comp v) { return enc(v); }
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
    // Raw domain: the FP32 number whose exponent and mantissa fields are the code's, i.e. the
    // value times 2^-120 (an FP32 denormal below 2^-6).  The bulk step works on raw values with
    // 2^120 folded into its constants: decoding is a shift and a mask, and encoding is one
    // integer rounding of the FP32 pattern for every magnitude (the denormal patterns continue
    // the normal ones with the same spacing).  A raw result below 2^-126 has been rounded to
    // FP32's denormal spacing (2^-29 in value units) before that, a 2^-30 effect on a 2^-19
    // rounding step.
    static constexpr bool has_raw = true;
    static constexpr double raw_unit = 0x1p-120;  // raw value = value * raw_unit
    __device__ static comp dec_raw(elem v) {
        const unsigned x = ((unsigned)v) << 16;
        return __uint_as_float(((x >> 5) & 0x03fff800u) | (x & 0x80000000u));
    }
    __device__ static elem enc_raw(comp v) {
        const unsigned bits = __float_as_uint(v);
        const unsigned b = bits & 0x7fffffffu;
        const unsigned code = min((b + 0x3ffu + ((b >> 11) & 1u)) >> 11, 0x7fffu);
        return (elem)(code | ((bits >> 16) & 0x8000u));
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

// Element decode/encode in the real or (RAW) raw domain.
template <class ST, bool RAW>
__device__ __forceinline__ typename ST::comp dec_io(typename ST::elem v) {
    if constexpr (RAW)
        return ST::dec_raw(v);
    else
        return ST::dec(v);
}
template <class ST, bool RAW>
__device__ __forceinline__ typename ST::elem enc_io(typename ST::comp v) {
    if constexpr (RAW)
        return ST::enc_raw(v);
    else
        return ST::enc(v);
}

template <class ST, bool RAW = false>
__device__ inline void load4(const typename ST::elem *p, typename ST::comp (&v)[4], bool nt = false) {
    using E = typename ST::elem;
    typedef E e4 __attribute__((ext_vector_type(4)));
    const e4 a = vload(reinterpret_cast<const e4 *>(p), nt);
    v[0] = dec_io<ST, RAW>(a.x);
    v[1] = dec_io<ST, RAW>(a.y);
    v[2] = dec_io<ST, RAW>(a.z);
    v[3] = dec_io<ST, RAW>(a.w);
}

template <class ST, bool RAW = false>
__device__ inline void store4(typename ST::elem *p, const typename ST::comp (&v)[4], bool nt = false) {
    using E = typename ST::elem;
    typedef E e4 __attribute__((ext_vector_type(4)));
    const e4 a = {enc_io<ST, RAW>(v[0]), enc_io<ST, RAW>(v[1]), enc_io<ST, RAW>(v[2]), enc_io<ST, RAW>(v[3])};
    vstore(reinterpret_cast<e4 *>(p), a, nt);
}

// Two consecutive elements starting at an even index: one 16-, 8- or 4-byte access.
template <class ST, bool RAW = false>
__device__ inline void load2(const typename ST::elem *p, typename ST::comp (&v)[2], bool nt = false) {
    using E = typename ST::elem;
    typedef E e2 __attribute__((ext_vector_type(2)));
    const e2 a = vload(reinterpret_cast<const e2 *>(p), nt);
    v[0] = dec_io<ST, RAW>(a.x);
    v[1] = dec_io<ST, RAW>(a.y);
}
template <class ST, bool RAW = false>
__device__ inline void store2(typename ST::elem *p, const typename ST::comp (&v)[2], bool nt = false) {
    using E = typename ST::elem;
    typedef E e2 __attribute__((ext_vector_type(2)));
    const e2 a = {enc_io<ST, RAW>(v[0]), enc_io<ST, RAW>(v[1])};
    vstore(reinterpret_cast<e2 *>(p), a, nt);
}

}  // namespace lbm
