// Split-BF16 kernels: the same arithmetic as the generic stage and fused kernels,
// organised for latency.  Operands shared by a workgroup (Phi and zeta in their three-term
// BF16 planes, zeta in FP32 for the Khatri-Rao factor, the eigenvalues) live in LDS for the
// whole launch -- all of them for systems of up to 64 states, a t-slice for larger ones;
// the grid is a few workgroups per CU that sweep the items, and the right operand rows of
// the next item are loaded into registers while the current item computes.
//
// This header holds what the four kernel files share (internal linkage in each).
#pragma once

#include <type_traits>

#include "npf_device.h"
#include "npf_internal.h"
#include "npf_mfma.h"

namespace npf {

constexpr int kBf3Threads = 256;

struct Bf3Args {
    const void *X;           // fused: T_{M-1} [U_{M-1}][n][Jpad]; stage: T_{i-1}
    void *out;               // stage: T_i
    const __bf16 *phiE;      // 6 planes [pl][a/8][t][a%8]
    const __bf16 *zetaE;     // 6 planes [pl][t/4][k][t%4]
    const float2 *zeta32;    // [npad][npad] delta Psi
    const double2 *lam;      // [n]
    const double2 *lamj;     // fused: eigenvalues of the computed modes (mode j0 + jl)
    const uint64_t *ptab;    // sorted prefixes (fused: length M-1; stage: length i-1)
    const uint64_t *stab;    // stage: sorted suffixes of length M-i
    double2 *parts;          // fused: [gridDim.x][Jpad][n]
    int64_t n, Jpad, J, j0, items, U_suf, U_in;
    int M, i;
    double eps, tau2;
};

// Position of a workgroup among the workgroups of its system.
struct BlockPos {
    int64_t x, gx;           // index along the items, and their number
    int y, z;
    int sys;
};

// Position along the items of workgroup b of a single-system launch of g workgroups: the
// workgroups are dealt to the eight XCDs in turn (b % 8), so with g a multiple of 8 each
// XCD is given a contiguous run of g / 8 starting items -- items that read common rows
// then meet in the same L2.
__device__ __forceinline__ int64_t xcd_block(unsigned b, unsigned g)
{
    return (g % 8u == 0u) ? int64_t(b % 8u) * (g / 8u) + b / 8u : int64_t(b);
}

// For a launch over several systems: system s owns workgroups [first[s], first[s+1]) of
// grid.x (every system at least one).
__device__ __forceinline__ BlockPos system_block(const int32_t *__restrict__ first, int nsys)
{
    const int32_t b = int32_t(blockIdx.x);
    int lo = 0, hi = nsys - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return BlockPos{b - first[lo], first[lo + 1] - first[lo], int(blockIdx.y), int(blockIdx.z), lo};
}

template <int NP>
__device__ __forceinline__ void copy_to_lds(char *dst, const void *src, int64_t bytes)
{
    const int4 *s = reinterpret_cast<const int4 *>(src);
    int4 *d = reinterpret_cast<int4 *>(dst);
    for (int64_t x = threadIdx.x; x < bytes / 16; x += blockDim.x) d[x] = s[x];
}

// A operand fragments of Phi^T (rows t0 + c, columns a0 + 8g .. +7) from the LDS planes.
template <int NP>
__device__ __forceinline__ void phi_frags(const __bf16 *L, int a0, int t, int g, Split3 &pr,
                                          Split3 &pi)
{
    constexpr int N2 = NP * NP;
    const int pidx = ((a0 / 8 + g) * NP + t) * 8;
    pr.h = *reinterpret_cast<const v8bf *>(L + 0 * N2 + pidx);
    pr.m = *reinterpret_cast<const v8bf *>(L + 1 * N2 + pidx);
    pr.l = *reinterpret_cast<const v8bf *>(L + 2 * N2 + pidx);
    pi.h = *reinterpret_cast<const v8bf *>(L + 3 * N2 + pidx);
    pi.m = *reinterpret_cast<const v8bf *>(L + 4 * N2 + pidx);
    pi.l = *reinterpret_cast<const v8bf *>(L + 5 * N2 + pidx);
}

__device__ __forceinline__ void split_x(const float2 (&x)[8], Split3 &xr, Split3 &xi)
{
    float re[8], im[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        re[s] = x[s].x;
        im[s] = x[s].y;
    }
    xr = split8(re);
    xi = split8(im);
}

template <typename K>
void set_lds_limit(K kernel, int bytes)
{
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

inline Bf3Args base_args(const npf_plan_s *p, char *ws, const double *lam)
{
    const int64_t N2 = p->npad * p->npad;
    char *base = ws + p->lay.phi;
    Bf3Args a{};
    a.phiE = reinterpret_cast<const __bf16 *>(base + 16 * N2);
    a.zetaE = reinterpret_cast<const __bf16 *>(base + 34 * N2);
    a.zeta32 = reinterpret_cast<const float2 *>(base + 50 * N2);
    a.lam = reinterpret_cast<const double2 *>(lam);
    a.lamj = a.lam;
    a.n = p->n;
    a.Jpad = p->Jpad;
    a.eps = p->prob.eps;
    a.tau2 = p->prob.tau * p->prob.tau;
    return a;
}

// Arguments of chain stage i (Alg. 2 steps 2-3) of order ca.M.
inline Bf3Args stage_args(const ChainArgs &ca, int i)
{
    const npf_plan_s &p = *ca.plan;
    const int M = ca.M;
    const uint64_t *tt = reinterpret_cast<const uint64_t *>(ca.ws + p.lay.ttab);
    Bf3Args a = base_args(&p, ca.ws, nullptr);
    a.X = ca.ws + p.lay.buf[(i - 1) % 2];
    a.out = ca.ws + p.lay.buf[i % 2];
    a.ptab = tt + p.tt.off[i - 1 > 0 ? i - 1 : 1];
    a.stab = tt + p.tt.off[M - i > 0 ? M - i : 1];
    a.U_suf = p.U[M - i];
    a.U_in = p.U[M - i + 1];
    a.items = p.U[i - 1] * p.U[M - i];
    a.M = M;
    a.i = i;
    return a;
}

// Arguments of the fused last stage of order M for the block of modes [j0, j0 + J).
inline Bf3Args fused_args(const npf_plan_s *p, int M, int64_t j0, int64_t J, const double *lam,
                          char *ws)
{
    Bf3Args a = base_args(p, ws, lam);
    a.lamj = reinterpret_cast<const double2 *>(lam_rows(p, lam, ws));
    a.X = ws + p->lay.buf[(M - 1) % 2];
    a.ptab = reinterpret_cast<const uint64_t *>(ws + p->lay.ttab) + p->tt.off[M - 1];
    a.parts = reinterpret_cast<double2 *>(ws + p->lay.parts);
    a.J = J;
    a.j0 = j0;
    a.items = p->U[M - 1];
    a.M = M;
    return a;
}

}  // namespace npf
