// MFMA building blocks for gfx950: operand types, the three arithmetic engines and the
// split of FP32 values into three BF16 terms.
//
// Lane layouts (64 lanes, g = lane / 16, c = lane % 16), measured on the device:
//   f64 16x16x4 : A[i=c][k=g], B[k=g][j=c], D reg r holds D[4r + g][c]
//   f32 16x16x4 : A[i=c][k=g], B[k=g][j=c], D reg r holds D[4g + r][c]
//   bf16 16x16x32: A[i=c][k=8g+s], B[k=8g+s][j=c] (s = 0..7), D reg r holds D[4g + r][c]
//
// The FP32 engine keeps its operands and stored intermediates in FP32 but forms the products
// exactly and accumulates them in FP64, on the FP64 matrix cores: with FP32 accumulation
// (one rounding per four products) a chain of contractions over 200 states lost up to
// 1.1e-6 relative in P, the whole margin of the mixed paths' bound.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace npf {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __bf16 v4bf __attribute__((ext_vector_type(4)));

enum class Eng { F64 = 0, F32 = 1, BF3 = 2 };

template <Eng E> struct EngT;
template <> struct EngT<Eng::F64> {
    using acc = v4d;
    using real = double;
    using cplx = double2;
    static constexpr int KS = 4;    // K per MFMA
    static constexpr int TC = 16;   // t per chunk of the fused kernel
};
template <> struct EngT<Eng::F32> {
    using acc = v4d;                // FP64 accumulation of exact FP32 x FP32 products
    using real = float;
    using cplx = float2;
    static constexpr int KS = 4;
    static constexpr int TC = 16;
};
template <> struct EngT<Eng::BF3> {
    using acc = v4f;
    using real = float;
    using cplx = float2;
    static constexpr int KS = 32;
    static constexpr int TC = 32;
};

// Row of the 16x16 output tile held in accumulator register r by lane group g.
template <Eng E> __device__ __forceinline__ int out_row(int r, int g)
{
    if constexpr (E == Eng::F64 || E == Eng::F32) return 4 * r + g;
    else return 4 * g + r;
}

__device__ __forceinline__ v4d mfma(double a, double b, v4d c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// FP32 operands into an FP64 accumulator: the product of two FP32 values is exact in FP64.
__device__ __forceinline__ v4d mfma(float a, float b, v4d c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(double(a), double(b), c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma(v8bf a, v8bf b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Three-term BF16 split of FP32 operands: x = hi + mid + lo up to 2^-24 |x|.
struct Split3 {
    v8bf h, m, l;
};

__device__ __forceinline__ void split3(float x, __bf16 &h, __bf16 &m, __bf16 &l)
{
    h = __bf16(x);
    const float r1 = x - float(h);
    m = __bf16(r1);
    const float r2 = r1 - float(m);
    l = __bf16(r2);
}

// a*b with both split: the six products whose size is at least 2^-16 of hi*hi; the three
// dropped ones (mid*lo, lo*mid, lo*lo) are below 2^-23 relative.
__device__ __forceinline__ v4f mm6(const Split3 &a, const Split3 &b, v4f c)
{
    c = mfma(a.h, b.l, c);
    c = mfma(a.l, b.h, c);
    c = mfma(a.m, b.m, c);
    c = mfma(a.h, b.m, c);
    c = mfma(a.m, b.h, c);
    c = mfma(a.h, b.h, c);
    return c;
}

// mm6 with the sum kept in two parts: the hi*hi product goes to `hi`, the five smaller
// products (at most 2^-7 of it) to `lo`.  A BF16 MFMA adds the exact sum of its products
// to the accumulator with one rounding to nearest, so `hi` takes one rounding per
// product pair instead of six and the roundings of `lo` are 2^-8 smaller; the caller
// forms hi + lo once at the end.
__device__ __forceinline__ void mm6s(const Split3 &a, const Split3 &b, v4f &hi, v4f &lo)
{
    lo = mfma(a.h, b.l, lo);
    lo = mfma(a.l, b.h, lo);
    lo = mfma(a.m, b.m, lo);
    lo = mfma(a.h, b.m, lo);
    lo = mfma(a.m, b.h, lo);
    hi = mfma(a.h, b.h, hi);
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Position of zeta[t][k] in a BF16 plane laid out so that the reduction's B fragment of
// lane (g, c) for the 32-row chunk t0 -- rows t0 + 4g + s (s < 4) and t0 + 16 + 4g + s - 4
// (s >= 4), the K-slot order implied by the first product's accumulator layout -- is one
// contiguous 16-byte vector.
__host__ __device__ __forceinline__ int64_t zeta_frag_index(int64_t t, int64_t k, int64_t npad)
{
    const int64_t chunk = t >> 5, tt = t & 31;
    const int64_t g = (tt & 15) >> 2, s = (tt & 3) + ((tt >> 4) << 2);
    return ((chunk * 4 + g) * npad + k) * 8 + s;
}

// Exact three-term split by truncation: hi = the top 8 significand bits of x, mid = the top
// 8 of the remainder, lo = the rest (at most 8 bits), so x = hi + mid + lo exactly for a
// normal FP32 x.  Two values are split and packed at once (x0 in the low half).
__device__ __forceinline__ void split_pair(float x0, float x1, unsigned &h, unsigned &m,
                                           unsigned &l)
{
    const unsigned b0 = __float_as_uint(x0), b1 = __float_as_uint(x1);
    const float r0 = x0 - __uint_as_float(b0 & 0xffff0000u);
    const float r1 = x1 - __uint_as_float(b1 & 0xffff0000u);
    const unsigned c0 = __float_as_uint(r0), c1 = __float_as_uint(r1);
    const float q0 = r0 - __uint_as_float(c0 & 0xffff0000u);
    const float q1 = r1 - __uint_as_float(c1 & 0xffff0000u);
    // v_perm_b32: bytes 2-3 of the second operand, then bytes 2-3 of the first.
    h = __builtin_amdgcn_perm(b1, b0, 0x07060302u);
    m = __builtin_amdgcn_perm(c1, c0, 0x07060302u);
    l = __builtin_amdgcn_perm(__float_as_uint(q1), __float_as_uint(q0), 0x07060302u);
}

// Split eight FP32 values into the three BF16 operand vectors.
__device__ __forceinline__ Split3 split8(const float (&x)[8])
{
    u32x4 h, m, l;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        unsigned a, b, c;
        split_pair(x[2 * q], x[2 * q + 1], a, b, c);
        h[q] = a;
        m[q] = b;
        l[q] = c;
    }
    return {__builtin_bit_cast(v8bf, h), __builtin_bit_cast(v8bf, m), __builtin_bit_cast(v8bf, l)};
}

__device__ __forceinline__ v8bf negx(v8bf v)
{
    u32x4 u = __builtin_bit_cast(u32x4, v);
    u ^= 0x80008000u;
    return __builtin_bit_cast(v8bf, u);
}

__device__ __forceinline__ Split3 negx3(const Split3 &a) { return {negx(a.h), negx(a.m), negx(a.l)}; }

__device__ __forceinline__ v8bf neg8(v8bf v)
{
    v8bf r;
#pragma unroll
    for (int s = 0; s < 8; ++s) r[s] = -v[s];
    return r;
}

__device__ __forceinline__ Split3 neg3(const Split3 &a) { return {neg8(a.h), neg8(a.m), neg8(a.l)}; }

}  // namespace npf
