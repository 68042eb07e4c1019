// Device helpers: packed symmetric index arithmetic and the FP64 divisor.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "npf.h"

namespace npf {

constexpr int kMaxOrder = NPF_MAX_ORDER;

// binom(x + i - 1, i) for x >= 0, i >= 1: the colex weight of value x at position i.
__host__ __device__ __forceinline__ int64_t colex_term(int64_t x, int i)
{
    int64_t r = x;
    for (int s = 1; s < i; ++s) r = r * (x + s) / (s + 1);
    return r;
}

// colex_term with constant divisors for the orders used here (i <= 6), x < 2^16.
__host__ __device__ __forceinline__ int64_t colex_term_c(int64_t x, int i)
{
    switch (i) {
    case 1: return x;
    case 2: return x * (x + 1) / 2;
    case 3: return x * (x + 1) * (x + 2) / 6;
    case 4: return x * (x + 1) * (x + 2) * (x + 3) / 24;
    case 5: return x * (x + 1) * (x + 2) * (x + 3) * (x + 4) / 120;
    default: return colex_term(x, i);
    }
}

// Entry A_M[k, r] of a hash-generated derivative tensor: SplitMix64 (Steele, Lea and Flood
// 2014) output number (M << 49 | k << 40 | r) from `seed`; the sum S of its four 16-bit
// fields gives ((S - 131070) 2^-16 sqrt(3)) scale, an Irwin-Hall variate of mean 0 and
// variance scale^2.  Integer work and two IEEE products: every device reproduces the bits.
__host__ __device__ __forceinline__ double hash_entry(uint64_t seed, double scale, int M,
                                                      int64_t k, int64_t r)
{
    const uint64_t idx = (uint64_t(M) << 49) | (uint64_t(k) << 40) | uint64_t(r);
    uint64_t z = seed + (idx + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const int s = int(z & 0xffffu) + int((z >> 16) & 0xffffu) + int((z >> 32) & 0xffffu) +
                  int(z >> 48);
    const double x = double(s - 131070) * 0x1p-16;
    const double y = x * 1.7320508075688772;
    return y * scale;
}

// Sorted tuples of length <= 7 over n <= 512 states are packed 9 bits per entry, entry i in
// bits [9i, 9i + 9).
constexpr int kTupleBits = 9;
constexpr uint64_t kTupleMask = (uint64_t(1) << kTupleBits) - 1;

__host__ __device__ __forceinline__ int32_t tuple_at(uint64_t pk, int i)
{
    return int32_t((pk >> (kTupleBits * i)) & kTupleMask);
}

__host__ __device__ __forceinline__ uint64_t tuple_entry(int32_t v, int i)
{
    return uint64_t(v) << (kTupleBits * i);
}

__host__ __device__ __forceinline__ void unpack_tuple(uint64_t pk, int m, int32_t *t)
{
    for (int i = 0; i < m; ++i) t[i] = tuple_at(pk, i);
}

// Colex rank of a sorted m-tuple.
__host__ __device__ __forceinline__ int64_t colex_rank(const int32_t *t, int m)
{
    int64_t r = 0;
    for (int i = 0; i < m; ++i) r += colex_term(t[i], i + 1);
    return r;
}

// Sorted m-tuple over [0, n) with colex rank r (binary search per position).
__host__ __device__ __forceinline__ void colex_unrank(int64_t r, int m, int64_t n, int32_t *t)
{
    for (int i = m; i >= 1; --i) {
        int64_t lo = 0, hi = n - 1;  // largest x with colex_term(x, i) <= r
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) / 2;
            if (colex_term_c(mid, i) <= r) lo = mid; else hi = mid - 1;
        }
        t[i - 1] = int32_t(lo);
        r -= colex_term_c(lo, i);
    }
}

// Advance a sorted m-tuple over [0, n) to its colex successor; false after the last.
__host__ __device__ __forceinline__ bool colex_next(int32_t *t, int m, int64_t n)
{
    for (int i = 0; i < m; ++i) {
        const int64_t cap = (i + 1 < m) ? t[i + 1] : n - 1;
        if (t[i] < cap) {
            t[i] += 1;
            for (int l = 0; l < i; ++l) t[l] = 0;
            return true;
        }
    }
    return false;
}

// Colex rank of sort({a} U s) for a sorted m-tuple s.
__host__ __device__ __forceinline__ int64_t colex_rank_insert(int32_t a, const int32_t *s, int m)
{
    int64_t r = 0;
    int pos = 1;
    bool placed = false;
    for (int i = 0; i < m; ++i) {
        if (!placed && a <= s[i]) {
            r += colex_term(a, pos++);
            placed = true;
        }
        r += colex_term(s[i], pos++);
    }
    if (!placed) r += colex_term(a, pos);
    return r;
}

// rank(sort({a} U s)) for a fixed sorted suffix s of length m, with the parts that do not
// depend on a precomputed: = lo[q] + colex_term(a, q + 1) + hi[q], q = #{l : s_l <= a}.
struct InsertRank {
    int m;
    int32_t s[NPF_MAX_ORDER];
    int64_t lo[NPF_MAX_ORDER + 1], hi[NPF_MAX_ORDER + 1];

    __host__ __device__ void init(const int32_t *s_, int m_)
    {
        m = m_;
        for (int l = 0; l < m; ++l) s[l] = s_[l];
        lo[0] = 0;
        for (int q = 1; q <= m; ++q) lo[q] = lo[q - 1] + colex_term_c(s[q - 1], q);
        hi[m] = 0;
        for (int q = m - 1; q >= 0; --q) hi[q] = hi[q + 1] + colex_term_c(s[q], q + 2);
    }
    __host__ __device__ int64_t rank(int32_t a) const
    {
        int q = 0;
        for (int l = 0; l < m; ++l) q += (s[l] <= a) ? 1 : 0;
        return lo[q] + colex_term_c(a, q + 1) + hi[q];
    }
};

// rank(sort({a} U s)) with s held in registers (no dynamically indexed arrays).
__host__ __device__ __forceinline__ int64_t rank_insert_reg(int32_t a,
                                                            const int32_t (&s)[NPF_MAX_ORDER],
                                                            int m)
{
    int64_t r = 0;
    int q = 0;
#pragma unroll
    for (int l = 0; l < NPF_MAX_ORDER; ++l) {
        if (l < m) {
            if (s[l] <= a) {
                r += colex_term_c(s[l], l + 1);
                ++q;
            } else {
                r += colex_term_c(s[l], l + 2);
            }
        }
    }
    return r + colex_term_c(a, q + 1);
}

// unpack_tuple into a fixed-size register array.
__host__ __device__ __forceinline__ void unpack_tuple_reg(uint64_t pk, int m,
                                                          int32_t (&t)[NPF_MAX_ORDER])
{
#pragma unroll
    for (int i = 0; i < NPF_MAX_ORDER; ++i) t[i] = (i < m) ? tuple_at(pk, i) : 0;
}

// Orderings of a sorted tuple: M! / prod(count_v!).
__host__ __device__ __forceinline__ double multiplicity(const int32_t *s, int M)
{
    double f = 1.0;
    for (int i = 2; i <= M; ++i) f *= double(i);
    int run = 1;
    double den = 1.0;
    for (int i = 1; i <= M; ++i) {
        if (i < M && s[i] == s[i - 1]) {
            ++run;
            den *= double(run);
        } else {
            run = 1;
        }
    }
    return f / den;
}

// Small divisor of Alg. 2 steps 5-9 in FP64: the eigenvalues of the sorted tuple are
// summed left to right, then lam_j is subtracted; if |D|^2 < eps^2 then D = eps.  No
// fused multiply-add, so every implementation that follows the same order rounds the
// same way near a resonance.
__device__ __forceinline__ double2 divisor_fp64(double2 acc, double2 lam_j, double eps)
{
#pragma clang fp contract(off)
    double re = acc.x - lam_j.x;
    double im = acc.y - lam_j.y;
    const double mag2 = re * re + im * im;
    if (mag2 < eps * eps) {
        re = eps;
        im = 0.0;
    }
    return make_double2(re, im);
}

__device__ __forceinline__ double2 add_fp64(double2 a, double2 b)
{
    return make_double2(a.x + b.x, a.y + b.y);
}

// (a + ib) / (c + id), plain formula in FP64.
__device__ __forceinline__ double2 cdiv(double2 a, double2 d)
{
    const double den = d.x * d.x + d.y * d.y;
    return make_double2((a.x * d.x + a.y * d.y) / den, (a.y * d.x - a.x * d.y) / den);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

}  // namespace npf
