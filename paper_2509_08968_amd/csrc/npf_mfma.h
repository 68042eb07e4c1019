// MFMA building blocks for gfx950: operand types, the three arithmetic engines and the
// split of FP32 values into three BF16 terms.
//
// Lane layouts (64 lanes, g = lane / 16, c = lane % 16), measured on the device:
//   f64 16x16x4 : A[i=c][k=g], B[k=g][j=c], D reg r holds D[4r + g][c]
//   f32 16x16x4 : A[i=c][k=g], B[k=g][j=c], D reg r holds D[4g + r][c]
//   bf16 16x16x32: A[i=c][k=8g+s], B[k=8g+s][j=c] (s = 0..7), D reg r holds D[4g + r][c]
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
    using acc = v4f;
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
    if constexpr (E == Eng::F64) return 4 * r + g;
    else return 4 * g + r;
}

__device__ __forceinline__ v4d mfma(double a, double b, v4d c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma(float a, float b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
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

__device__ __forceinline__ v8bf neg8(v8bf v)
{
    v8bf r;
#pragma unroll
    for (int s = 0; s < 8; ++s) r[s] = -v[s];
    return r;
}

__device__ __forceinline__ Split3 neg3(const Split3 &a) { return {neg8(a.h), neg8(a.m), neg8(a.l)}; }

}  // namespace npf
