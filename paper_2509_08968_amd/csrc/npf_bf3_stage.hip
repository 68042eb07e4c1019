// Split-BF16 chain stage for systems of up to 64 states.
#include "npf_bf3.h"

namespace npf {

namespace {

constexpr int kThreads = kBf3Threads;

// ------------------------------------------------------------------ one chain stage
template <int NP, int SUF>
__device__ __forceinline__ void stage_bf3_body(const Bf3Args &a, const BlockPos bp)
{
    constexpr int NTT = NP / 16, KC = NP / 32;
    extern __shared__ __align__(16) char lds[];
    __shared__ int32_t sidx[2][NP];
    __shared__ int64_t rowoff[NP];      // binom(t + i - 1, i) * U_suf * Jpad
    const __bf16 *Lphi = reinterpret_cast<const __bf16 *>(lds);
    copy_to_lds<NP>(lds, a.phiE, 12 * NP * NP);
    for (int t = threadIdx.x; t < NP; t += blockDim.x)
        rowoff[t] = colex_term_c(t, a.i) * a.U_suf * a.Jpad;

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int64_t jw = int64_t(bp.y) * 64 + wave * 16;
    const bool wave_on = jw < a.Jpad;
    const float2 *X = static_cast<const float2 *>(a.X);

    auto build_idx = [&](int64_t it, int buf) {
        const int64_t rs = it % a.U_suf;
        const uint64_t pk = a.stab[rs];
        if (threadIdx.x < a.n) {
            // rank(sort({x} U s)) for the sorted suffix s (SUF entries, in registers).
            const int32_t x = int32_t(threadIdx.x);
            int64_t r = 0;
            int qq = 0;
#pragma unroll
            for (int l = 0; l < SUF; ++l) {
                const int32_t sl = tuple_at(pk, l);
                if (sl <= x) {
                    r += colex_term_c(sl, l + 1);
                    ++qq;
                } else {
                    r += colex_term_c(sl, l + 2);
                }
            }
            sidx[buf][threadIdx.x] = int32_t(r + colex_term_c(x, qq + 1));
        }
    };
    float2 xn[KC][8];
    auto gather_x = [&](int64_t it, int buf) {
        const int64_t rp = it / a.U_suf;
        const float2 *src = X + rp * a.U_in * a.Jpad + jw + c;
        const unsigned jp = unsigned(a.Jpad);
        const int nn = int(a.n);
#pragma unroll
        for (int kc = 0; kc < KC; ++kc)
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int ar = kc * 32 + 8 * g + s;
                xn[kc][s] = ar < nn ? src[uint64_t(unsigned(sidx[buf][ar])) * jp]
                                    : make_float2(0.f, 0.f);
            }
    };

    int64_t it = bp.x;
    int buf = 0;
    if (it < a.items) build_idx(it, 0);
    __syncthreads();          // also orders the LDS copy of Phi
    if (it < a.items && wave_on) gather_x(it, 0);
    for (; it < a.items; it += bp.gx, buf ^= 1) {
        Split3 xr[KC], xi[KC], xn_[KC];
        // Chunks of 32 gathered rows that are zero across the wave add nothing to the
        // products and are skipped (block-sparse tensors leave most of them zero in the
        // first stages: a row is nonzero only if its states share a support block).
        int live = 0;
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            bool nz = false;
#pragma unroll
            for (int s = 0; s < 8; ++s) nz = nz || xn[kc][s].x != 0.f || xn[kc][s].y != 0.f;
            if (__any(nz)) live |= 1 << kc;
            split_x(xn[kc], xr[kc], xi[kc]);
            xn_[kc] = negx3(xi[kc]);
        }
        const int64_t itn = it + bp.gx;
        if (itn < a.items) build_idx(itn, buf ^ 1);
        __syncthreads();
        if (itn < a.items && wave_on) gather_x(itn, buf ^ 1);
        if (!wave_on) continue;

        const int64_t rp = it / a.U_suf, rs = it % a.U_suf;
        int m = 0;
        if (a.i > 1) m = int(tuple_at(a.ptab[rp], a.i - 2));
        const int tt0 = m / 16;

        v4f sr[NTT], si[NTT], srl[NTT], sil[NTT];
#pragma unroll
        for (int tt = 0; tt < NTT; ++tt) sr[tt] = si[tt] = srl[tt] = sil[tt] = v4f{0, 0, 0, 0};
#pragma unroll
        for (int tt = 0; tt < NTT; ++tt) {
            if (tt < tt0) continue;
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
                if (!((live >> kc) & 1)) continue;
                Split3 pr, pi;
                phi_frags<NP>(Lphi, kc * 32, tt * 16 + c, g, pr, pi);
                mm6s(pr, xr[kc], sr[tt], srl[tt]);
                mm6s(pi, xn_[kc], sr[tt], srl[tt]);
                mm6s(pr, xi[kc], si[tt], sil[tt]);
                mm6s(pi, xr[kc], si[tt], sil[tt]);
            }
        }
        // Row rank(p U t) = rp + binom(t + i - 1, i).
        float2 *dst = static_cast<float2 *>(a.out) + (rp * a.U_suf + rs) * a.Jpad + jw + c;
        const int nn = int(a.n);
#pragma unroll
        for (int tt = 0; tt < NTT; ++tt) {
            if (tt < tt0) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int t = tt * 16 + 4 * g + r;
                if (t < m || t >= nn) continue;
                dst[rowoff[t]] = make_float2(sr[tt][r] + srl[tt][r], si[tt][r] + sil[tt][r]);
            }
        }
    }
}

// Two workgroups per CU: the register budget is held to 256 per lane.
template <int NP, int SUF>
__global__ void __launch_bounds__(kThreads, 2)
stage_bf3(Bf3Args a)
{
    stage_bf3_body<NP, SUF>(a, BlockPos{xcd_block(blockIdx.x, gridDim.x), gridDim.x, int(blockIdx.y), int(blockIdx.z), 0});
}

// The same for several systems in one launch: workgroups [first[s], first[s+1]) of grid.x
// run system s with the arguments as[s].
template <int NP, int SUF>
__global__ void __launch_bounds__(kThreads, 2)
stage_bf3_multi(const Bf3Args *__restrict__ as, const int32_t *__restrict__ first, int nsys)
{
    const BlockPos bp = system_block(first, nsys);
    stage_bf3_body<NP, SUF>(as[bp.sys], bp);
}

}  // namespace

hipError_t launch_stage_bf3_small(const ChainArgs &ca, int i)
{
    const npf_plan_s &p = *ca.plan;
    const Bf3Args a = stage_args(ca, i);
    const int suf = ca.M - i;
    const int64_t jgroups = (p.Jpad + 63) / 64;
    int64_t groups = 512 / jgroups;
    if (groups > a.items) groups = a.items;
    if (groups >= 64) groups -= groups % 8;       // whole XCD rounds (xcd_block)
    if (groups < 1) groups = 1;
    const dim3 grid{unsigned(groups), unsigned(jgroups), 1u};
    const size_t shm = size_t(12 * p.npad * p.npad);
#define NPF_STAGE_CASE(NP_, S_)                                                           \
    if (p.npad == NP_ && suf == S_) {                                                    \
        set_lds_limit(stage_bf3<NP_, S_>, int(shm));                                      \
        hipLaunchKernelGGL((stage_bf3<NP_, S_>), grid, dim3(kThreads), shm, ca.stream, a); \
        return hipGetLastError();                                                         \
    }
    NPF_STAGE_CASE(32, 1) NPF_STAGE_CASE(32, 2) NPF_STAGE_CASE(32, 3)
    NPF_STAGE_CASE(64, 1) NPF_STAGE_CASE(64, 2) NPF_STAGE_CASE(64, 3)
#undef NPF_STAGE_CASE
    return hipErrorInvalidValue;
}

bool bf3_stage_supported(const npf_plan_s *p)
{
    return p->prec == NPF_BF16X3 && p->N <= 4;
}

hipError_t launch_stage_bf3_multi(int npad, int suf, const MultiLaunch &m)
{
    const dim3 grid{unsigned(m.groups), unsigned(m.gy), 1u};
    const size_t shm = size_t(12 * npad * npad);
    const Bf3Args *as = static_cast<const Bf3Args *>(m.args);
#define NPF_STAGE_MULTI(NP_, S_)                                                           \
    if (npad == NP_ && suf == S_) {                                                       \
        set_lds_limit(stage_bf3_multi<NP_, S_>, int(shm));                                 \
        hipLaunchKernelGGL((stage_bf3_multi<NP_, S_>), grid, dim3(kThreads), shm, m.stream, \
                           as, m.first, m.nsys);                                           \
        return hipGetLastError();                                                          \
    }
    NPF_STAGE_MULTI(32, 1) NPF_STAGE_MULTI(32, 2) NPF_STAGE_MULTI(32, 3)
    NPF_STAGE_MULTI(64, 1) NPF_STAGE_MULTI(64, 2) NPF_STAGE_MULTI(64, 3)
#undef NPF_STAGE_MULTI
    return hipErrorInvalidValue;
}

}  // namespace npf
