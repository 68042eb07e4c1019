// Derivative tensors of a polynomial vector field at the expansion point x*, from
// evaluations of the field: the numerical Taylor expansion that produces the tensors of
// Alg. 1, one batch of rows (an index range over the outermost dimension) per call.
//
// Entry (k, t) of A_M, t = (t_1 <= .. <= t_M), is the mixed derivative of f_k by
// x_{t_1} .. x_{t_M} at x*.  Two exact steps give it from values of f_k:
//   * polarization: for a form g homogeneous of degree M,
//       sum over the subsets S of [M] of (-1)^(M - |S|) g(y_S),  y_S = sum_{i in S} e_{t_i},
//     is that derivative, and the same alternating sum annihilates every form of degree
//     < M (as a function of the indicators of S it has no term in all M of them);
//   * the part of degree exactly M is the coefficient of s^M in the polynomial
//       p(s) = sum_S (-1)^(M - |S|) f_k(x* + s y_S),
//     whose other coefficients are those of degrees M+1 .. d for a term of degree d, so
//     d - M + 1 values of p at the nonzero nodes 1, -1, 2, -2, .. fix it by Lagrange
//     interpolation of p(s) / s^M at s = 0.
// Both steps are exact for polynomials, so the result differs from the derivative only by
// rounding.  The field is evaluated term by term, so that each monomial uses the nodes its
// own degree needs; a term of degree below M contributes nothing and is skipped, and at
// x* = 0 so is every term whose degree is not M (its expansion has no part of degree M),
// as is the empty subset (every term vanishes at y = 0 there).
#include <cmath>
#include <string>

#include "npf_device.h"
#include "npf_internal.h"

namespace npf {

namespace {

constexpr int kTaylorThreads = 256;
constexpr int kMaxDegree = 8;

// Node e of the interpolation: 1, -1, 2, -2, 3, ...
__device__ __forceinline__ double node(int e) { return (e & 1) ? -double(e / 2 + 1) : double(e / 2 + 1); }

// Weight of p(s_e) in the coefficient of s^M of a polynomial of degrees M .. M + m - 1
// from its values at the first m nodes: L_e(0) / s_e^M with L_e the Lagrange basis
// polynomial.  Numerator and denominator are products of small integers (exact in FP64),
// so the weight takes one rounding.
__device__ __forceinline__ double node_weight(int e, int m, int M)
{
    const double se = node(e);
    double num = 1.0, den = 1.0;
    for (int f = 0; f < m; ++f) {
        if (f == e) continue;
        const double sf = node(f);
        num *= -sf;
        den *= se - sf;
    }
    for (int i = 0; i < M; ++i) den *= se;
    return num / den;
}

// One workgroup per (row k, range of kTaylorThreads ranks).  The row's terms are read in
// rounds of kTaylorThreads, one per thread; the ones that can contribute (degree >= M, and at
// x* = 0 degree exactly M) are compacted into LDS in their original order -- a prefix sum of
// the per-wave ballots, so the order of the sums is fixed -- and every thread then evaluates
// its entry over them.
template <int M>
__global__ __launch_bounds__(kTaylorThreads) void taylor_fill(
    int64_t n, int64_t k0, int64_t rows, int64_t UM, const int64_t *__restrict__ eq_ptr,
    int64_t n_terms, const double *__restrict__ coef, const int32_t *__restrict__ var, int D,
    const double *__restrict__ x_eq, double *__restrict__ out)
{
    constexpr int NW = kTaylorThreads / 64;
    __shared__ double s_coef[kTaylorThreads];
    __shared__ int32_t s_var[kTaylorThreads][kMaxDegree];
    __shared__ int32_t s_deg[kTaylorThreads];
    __shared__ int s_wcnt[NW];
    __shared__ int s_bad;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t r = int64_t(blockIdx.x) * kTaylorThreads + threadIdx.x;
    const bool live = r < UM;
    int32_t t[M];
    if (live) colex_unrank(r, M, n, t);
    else
        for (int l = 0; l < M; ++l) t[l] = 0;
    for (int64_t kr = blockIdx.y; kr < rows; kr += gridDim.y) {
        const int64_t k = k0 + kr;
        int64_t q0 = eq_ptr[k], q1 = eq_ptr[k + 1];
        q0 = q0 < 0 ? 0 : (q0 > n_terms ? n_terms : q0);
        q1 = q1 < q0 ? q0 : (q1 > n_terms ? n_terms : q1);
        if (threadIdx.x == 0) s_bad = 0;
        __syncthreads();              // reset before any thread can flag this row
        double acc = 0.0;
        for (int64_t qb = q0; qb < q1; qb += kTaylorThreads) {
            // Stage this round's contributing terms.
            const int64_t q = qb + threadIdx.x;
            int32_t a[kMaxDegree];
            int d = 0;
            bool keep = false;
            if (q < q1) {
#pragma unroll
                for (int i = 0; i < kMaxDegree; ++i) {
                    a[i] = i < D ? var[q * D + i] : -1;
                    if (a[i] >= n) s_bad = 1;
                    if (a[i] < 0 || a[i] >= n) a[i] = -1;
                    else ++d;
                }
                keep = d >= M && (x_eq || d == M);
            }
            const uint64_t bal = __ballot(keep);
            if (lane == 0) s_wcnt[wave] = __popcll(bal);
            __syncthreads();
            int base = 0, total = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                base += w < wave ? s_wcnt[w] : 0;
                total += s_wcnt[w];
            }
            if (keep) {
                const int slot = base + __popcll(bal & ((uint64_t(1) << lane) - 1));
                s_coef[slot] = coef[q];
                s_deg[slot] = d;
                int m = 0;
#pragma unroll
                for (int i = 0; i < kMaxDegree; ++i)
                    if (a[i] >= 0) s_var[slot][m++] = a[i];
            }
            __syncthreads();
            if (live) {
                for (int u = 0; u < total; ++u) {
                    const int du = s_deg[u];
                    // The term's variables and, per variable, the positions of t holding it
                    // (a bit mask): y_S of that variable is popcount(mask & S).
                    int32_t v[kMaxDegree];
                    unsigned pos[kMaxDegree];
                    bool vanish = false;
#pragma unroll
                    for (int i = 0; i < kMaxDegree; ++i) {
                        v[i] = i < du ? s_var[u][i] : -1;
                        unsigned mk = 0;
#pragma unroll
                        for (int l = 0; l < M; ++l) mk |= unsigned(t[l] == v[i]) << l;
                        pos[i] = mk;
                        vanish |= i < du && mk == 0;
                    }
                    if (!x_eq && vanish) continue;
                    const double c = s_coef[u];
                    const int m = du - M + 1;
                    for (int e = 0; e < m; ++e) {
                        const double sn = node(e);
                        double pe = 0.0;
                        for (unsigned S = x_eq ? 0u : 1u; S < (1u << M); ++S) {
                            double prod = c;
#pragma unroll
                            for (int i = 0; i < kMaxDegree; ++i) {
                                if (i >= du) continue;
                                const double y = double(__popc(pos[i] & S));
                                prod *= x_eq ? fma(sn, y, x_eq[v[i]]) : sn * y;
                            }
                            pe += ((M - __popc(S)) & 1) ? -prod : prod;
                        }
                        acc = fma(node_weight(e, m, M), pe, acc);
                    }
                }
            }
            __syncthreads();          // the staged terms are rewritten next round
        }
        __syncthreads();              // every flag of this row is set
        if (live) out[kr * UM + r] = s_bad ? __builtin_nan("") : acc;
        __syncthreads();              // s_bad is read before the next row resets it
    }
}

template <int M>
hipError_t launch_taylor(int64_t n, int64_t k0, int64_t rows, int64_t UM, const npf_poly &p,
                         double *out, hipStream_t s)
{
    // Every rank has its thread (the workgroups stage the row's terms together); U_M < 2^40
    // and an output that fits the device keep bx far below the grid limit.
    const int64_t bx = (UM + kTaylorThreads - 1) / kTaylorThreads;
    if (bx > 0x7fffffff) return hipErrorInvalidConfiguration;
    const dim3 grid(unsigned(bx), unsigned(rows < 65535 ? rows : 65535));
    hipLaunchKernelGGL(taylor_fill<M>, grid, dim3(kTaylorThreads), 0, s, n, k0, rows, UM,
                       p.eq_ptr, p.n_terms, p.coef, p.var, int(p.max_degree), p.x_eq, out);
    return hipGetLastError();
}

}  // namespace

}  // namespace npf

extern "C" int npf_taylor_fill(int64_t n, int32_t order, const npf_poly *poly, int64_t k0,
                               int64_t k1, double *out, void *stream)
{
    using namespace npf;
    if (!poly) return fail(NPF_E_INVALID, "null polynomial field");
    if (n < 1) return fail(NPF_E_INVALID, "n < 1");
    if (order < 1 || order > NPF_MAX_ORDER) return fail(NPF_E_INVALID, "order outside [1, 6]");
    if (poly->max_degree < 1 || poly->max_degree > kMaxDegree)
        return fail(NPF_E_INVALID, "max_degree outside [1, 8]");
    if (poly->n_terms < 0) return fail(NPF_E_INVALID, "negative term count");
    if (k0 < 0 || k1 > n || k0 > k1) return fail(NPF_E_INVALID, "row range outside [0, n]");
    const int64_t UM = binom(n + order - 1, order);
    if (UM <= 0 || UM >= (int64_t(1) << 40)) return fail(NPF_E_INVALID, "U_M >= 2^40");
    if (k1 == k0) return NPF_OK;
    if (!out || !poly->eq_ptr) return fail(NPF_E_INVALID, "null output or eq_ptr");
    if (poly->n_terms > 0 && (!poly->coef || !poly->var))
        return fail(NPF_E_INVALID, "terms without coefficients or variables");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipErrorInvalidValue;
    switch (order) {
    case 1: e = launch_taylor<1>(n, k0, k1 - k0, UM, *poly, out, s); break;
    case 2: e = launch_taylor<2>(n, k0, k1 - k0, UM, *poly, out, s); break;
    case 3: e = launch_taylor<3>(n, k0, k1 - k0, UM, *poly, out, s); break;
    case 4: e = launch_taylor<4>(n, k0, k1 - k0, UM, *poly, out, s); break;
    case 5: e = launch_taylor<5>(n, k0, k1 - k0, UM, *poly, out, s); break;
    default: e = launch_taylor<6>(n, k0, k1 - k0, UM, *poly, out, s); break;
    }
    if (e != hipSuccess) return fail(NPF_E_DEVICE, std::string("taylor_fill: ") + hipGetErrorString(e));
    return NPF_OK;
}
