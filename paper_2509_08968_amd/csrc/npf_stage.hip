// One stage of the lower-index chain on MFMA (Alg. 2 steps 2-3, one mode product each):
//   T_i[rank(p U t)][rs][j] = sum_a T_{i-1}[rp][rank(sort(a U s))][j] Phi[a][t],  t >= last(p)
// for every sorted mode prefix p (length i-1, rank rp) and sorted state suffix s (length
// M-i, rank rs).  Per (p, s) item this is a [t x a] x [a x j] complex product whose right
// operand rows are gathered from the symmetric storage of T_{i-1}; the gather table
// rank(sort(a U s)) is built once per item in LDS.  Wave w of a workgroup owns 16 modes;
// every wave sweeps all t tiles of the item so each gathered row is read once.
#include "npf_device.h"
#include "npf_internal.h"
#include "npf_mfma.h"

namespace npf {

namespace {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kMaxN = 256;          // states supported by the MFMA chain kernels

struct StageArgs {
    const void *in;        // T_{i-1}: [U_{i-1}][U_in][Jpad]
    void *out;             // T_i:     [U_i][U_suf][Jpad]
    const void *phiE;      // staged Phi (engine layout)
    int64_t n, npad, Jpad, U_suf, U_in, items;
    int M, i;
};

template <Eng E, int NTT>
__global__ void __launch_bounds__(kThreads)
stage_mfma(StageArgs a)
{
    using T = EngT<E>;
    using acc_t = typename T::acc;
    using real = typename T::real;
    using cplx = typename T::cplx;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int64_t jw = int64_t(blockIdx.y) * 64 + wave * 16;
    const bool wave_on = jw < a.Jpad;
    const int ntt = int(a.npad / 16);

    __shared__ int32_t sidx[kMaxN];
    __shared__ int32_t sp[kMaxOrder], ss[kMaxOrder];
    __shared__ int64_t sbase;
    __shared__ int32_t sm;

    const int sufl = a.M - a.i;       // suffix length
    for (int64_t it = blockIdx.x; it < a.items; it += gridDim.x) {
        const int64_t rp = it / a.U_suf, rs = it % a.U_suf;
        __syncthreads();
        if (threadIdx.x == 0) {
            colex_unrank(rp, a.i - 1, a.n, sp);
            colex_unrank(rs, sufl, a.n, ss);
            sm = (a.i > 1) ? sp[a.i - 2] : 0;
            sbase = (a.i > 1) ? colex_rank(sp, a.i - 1) : 0;
        }
        __syncthreads();
        for (int x = threadIdx.x; x < a.n; x += blockDim.x)
            sidx[x] = int32_t(colex_rank_insert(int32_t(x), ss, sufl));
        __syncthreads();
        if (!wave_on) continue;
        const int m = sm;
        const int tt0 = m / 16;
        const cplx *src = static_cast<const cplx *>(a.in) + rp * a.U_in * a.Jpad + jw + c;

        acc_t sr[NTT], si[NTT];
#pragma unroll
        for (int tt = 0; tt < NTT; ++tt) sr[tt] = si[tt] = acc_t{0, 0, 0, 0};

        if constexpr (E != Eng::BF3) {
            const cplx *Ph = static_cast<const cplx *>(a.phiE);
            for (int64_t a0 = 0; a0 < a.npad; a0 += 4) {
                const int64_t ar = a0 + g;
                cplx x;
                if (ar < a.n) x = src[int64_t(sidx[ar]) * a.Jpad];
                else x = cplx{0, 0};
#pragma unroll
                for (int tt = 0; tt < NTT; ++tt) {
                    if (tt < tt0 || tt >= ntt) continue;
                    const cplx ph = Ph[ar * a.npad + tt * 16 + c];
                    sr[tt] = mfma(ph.x, x.x, sr[tt]);
                    sr[tt] = mfma(real(-ph.y), x.y, sr[tt]);
                    si[tt] = mfma(ph.x, x.y, si[tt]);
                    si[tt] = mfma(ph.y, x.x, si[tt]);
                }
            }
        } else {
            const __bf16 *Ph = static_cast<const __bf16 *>(a.phiE);
            const int64_t plane = a.npad * a.npad;
            for (int64_t a0 = 0; a0 < a.npad; a0 += 32) {
                Split3 xr, xi;
#pragma unroll
                for (int s = 0; s < 8; ++s) {
                    const int64_t ar = a0 + 8 * g + s;
                    float2 x = make_float2(0.f, 0.f);
                    if (ar < a.n) x = src[int64_t(sidx[ar]) * a.Jpad];
                    __bf16 h, mm, l;
                    split3(x.x, h, mm, l);
                    xr.h[s] = h; xr.m[s] = mm; xr.l[s] = l;
                    split3(x.y, h, mm, l);
                    xi.h[s] = h; xi.m[s] = mm; xi.l[s] = l;
                }
#pragma unroll
                for (int tt = 0; tt < NTT; ++tt) {
                    if (tt < tt0 || tt >= ntt) continue;
                    const int64_t pidx = ((a0 / 8 + g) * a.npad + tt * 16 + c) * 8;
                    Split3 pr, pi;
                    pr.h = *reinterpret_cast<const v8bf *>(Ph + 0 * plane + pidx);
                    pr.m = *reinterpret_cast<const v8bf *>(Ph + 1 * plane + pidx);
                    pr.l = *reinterpret_cast<const v8bf *>(Ph + 2 * plane + pidx);
                    pi.h = *reinterpret_cast<const v8bf *>(Ph + 3 * plane + pidx);
                    pi.m = *reinterpret_cast<const v8bf *>(Ph + 4 * plane + pidx);
                    pi.l = *reinterpret_cast<const v8bf *>(Ph + 5 * plane + pidx);
                    const Split3 pn = neg3(pi);
                    sr[tt] = mm6(pr, xr, sr[tt]);
                    sr[tt] = mm6(pn, xi, sr[tt]);
                    si[tt] = mm6(pr, xi, si[tt]);
                    si[tt] = mm6(pi, xr, si[tt]);
                }
            }
        }
        // Store T_i rows (p U t, s) for t >= m.
        const int64_t base = sbase;
        cplx *dst = static_cast<cplx *>(a.out) + rs * a.Jpad + jw + c;
#pragma unroll
        for (int tt = 0; tt < NTT; ++tt) {
            if (tt < tt0 || tt >= ntt) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t t = int64_t(tt) * 16 + out_row<E>(r, g);
                if (t < m || t >= a.n) continue;
                const int64_t row = base + colex_term(t, a.i);
                dst[row * a.U_suf * a.Jpad] = cplx{sr[tt][r], si[tt][r]};
            }
        }
    }
}

template <Eng E>
hipError_t launch_stage_eng(const StageArgs &sa, int ntt, int64_t groups, int64_t jgroups,
                            hipStream_t s)
{
    const dim3 grid{unsigned(groups), unsigned(jgroups), 1u};
    switch (ntt) {
    case 2: hipLaunchKernelGGL((stage_mfma<E, 2>), grid, dim3(kThreads), 0, s, sa); break;
    case 4: hipLaunchKernelGGL((stage_mfma<E, 4>), grid, dim3(kThreads), 0, s, sa); break;
    case 6: hipLaunchKernelGGL((stage_mfma<E, 6>), grid, dim3(kThreads), 0, s, sa); break;
    case 8: hipLaunchKernelGGL((stage_mfma<E, 8>), grid, dim3(kThreads), 0, s, sa); break;
    case 10: hipLaunchKernelGGL((stage_mfma<E, 10>), grid, dim3(kThreads), 0, s, sa); break;
    case 12: hipLaunchKernelGGL((stage_mfma<E, 12>), grid, dim3(kThreads), 0, s, sa); break;
    case 14: hipLaunchKernelGGL((stage_mfma<E, 14>), grid, dim3(kThreads), 0, s, sa); break;
    case 16: hipLaunchKernelGGL((stage_mfma<E, 16>), grid, dim3(kThreads), 0, s, sa); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

bool stage_mfma_supported(const npf_plan_s *p) { return p->n <= kMaxN; }

hipError_t launch_stage_mfma(const ChainArgs &ca, int i)
{
    const npf_plan_s &p = *ca.plan;
    const int M = ca.M;
    StageArgs sa;
    sa.in = ca.ws + p.lay.buf[(i - 1) % 2];
    sa.out = ca.ws + p.lay.buf[i % 2];
    sa.phiE = ca.ws + p.lay.phi + 16 * p.npad * p.npad;
    sa.n = p.n;
    sa.npad = p.npad;
    sa.Jpad = p.Jpad;
    sa.U_suf = p.U[M - i];
    sa.U_in = p.U[M - i + 1];
    sa.items = p.U[i - 1] * p.U[M - i];
    sa.M = M;
    sa.i = i;
    const int ntt = int(p.npad / 16);
    const int64_t jgroups = (p.Jpad + 63) / 64;
    int64_t groups = 8192 / jgroups;
    if (groups > sa.items) groups = sa.items;
    if (groups < 1) groups = 1;
    switch (p.prec) {
    case NPF_FP64: return launch_stage_eng<Eng::F64>(sa, ntt, groups, jgroups, ca.stream);
    case NPF_FP32: return launch_stage_eng<Eng::F32>(sa, ntt, groups, jgroups, ca.stream);
    default: return launch_stage_eng<Eng::BF3>(sa, ntt, groups, jgroups, ca.stream);
    }
}

}  // namespace npf
