// Split-BF16 fused last stage for systems of up to 64 states.
#include "npf_bf3.h"

namespace npf {

namespace {

constexpr int kThreads = 512;              // eight waves

// ------------------------------------------------------------------ fused last stage
// Eight waves: wave w owns the 16 modes of j-tile w % 4 and half h = w / 4 of the work --
// the 16-row t-tile h of each 32-row chunk in the first product, the k-tiles of half h in
// the reduction.  The two halves of a chunk's h meet in LDS (one barrier per chunk, the
// exchange buffer alternating), so no product is computed twice and each wave holds half of
// the reduction's accumulators: two waves per SIMD fit in the register file.
template <int NP, int M>
__device__ __forceinline__ void fused_bf3_body(const Bf3Args &a, const BlockPos bp)
{
    constexpr int NKT = NP / 16, KC = NP / 32, N2 = NP * NP;
    constexpr int KTW = NKT / 2;           // k-tiles per wave
    extern __shared__ __align__(16) char lds[];
    __bf16 *Lphi = reinterpret_cast<__bf16 *>(lds);
    __bf16 *Lz = reinterpret_cast<__bf16 *>(lds + 12 * N2);
    double2 *Llam = reinterpret_cast<double2 *>(lds + 24 * N2);
    float2 *Lx = reinterpret_cast<float2 *>(lds + 24 * N2 + 16 * NP);   // [2][4][2][4][64]
    copy_to_lds<NP>(lds, a.phiE, 12 * N2);
    copy_to_lds<NP>(lds + 12 * N2, a.zetaE, 12 * N2);
    for (int t = threadIdx.x; t < NP; t += blockDim.x)
        Llam[t] = t < a.n ? a.lam[t] : make_double2(0.0, 0.0);
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int jt = wave & 3, half = wave >> 2;
    const int g = lane >> 4, c = lane & 15;
    const int64_t jw = int64_t(bp.y) * 64 + jt * 16;
    const bool wave_on = jw < a.Jpad;
    const int64_t jl = jw + c;
    const bool j_ok = wave_on && jl < a.J;
    const double2 lam_j = j_ok ? a.lamj[a.j0 + jl] : make_double2(0.0, 0.0);
    // Below this |D|^2 (FP32) the divisor is finished in FP64: the tau band, and a margin
    // around eps so that the clamp is decided in FP64 exactly as specified.
    const float guard = fmaxf(float(a.tau2), float(4.0 * a.eps * a.eps));
    const int nn = int(a.n), jp = int(a.Jpad);

    double pacc_r[KTW][4], pacc_i[KTW][4];
#pragma unroll
    for (int kk = 0; kk < KTW; ++kk)
#pragma unroll
        for (int r = 0; r < 4; ++r) pacc_r[kk][r] = pacc_i[kk][r] = 0.0;

    const float2 *X = static_cast<const float2 *>(a.X);
    // The item's rows in FP32 (rows a >= n read row n - 1: the Phi planes are zero there).
    // The next item's prefix is loaded when an item starts, its rows once the item's first
    // products have split the current ones.
    float2 xv[KC][8];
    auto load_rows = [&](int64_t it) {
        const float2 *Xp = X + it * a.n * a.Jpad + jw + c;
#pragma unroll
        for (int kc = 0; kc < KC; ++kc)
#pragma unroll
            for (int s = 0; s < 8; ++s) xv[kc][s] = Xp[min(kc * 32 + 8 * g + s, nn - 1) * jp];
    };
    int buf = 0;
    uint64_t pk = 0, pkn = 0;
    if (int64_t(bp.x) < a.items) {
        pk = a.ptab[bp.x];
        if (wave_on) load_rows(bp.x);
    }
    // Items are the same for all eight waves (the barriers below are workgroup-uniform).
    for (int64_t it = bp.x; it < a.items; it += bp.gx, pk = pkn) {
        const int64_t itn = it + bp.gx;
        pkn = (itn < a.items) ? a.ptab[itn] : 0;
        int32_t p[M - 1];
#pragma unroll
        for (int q = 0; q < M - 1; ++q) p[q] = tuple_at(pk, q);
        double2 lam_p = Llam[p[0]];
        double den = 1.0;
        int run = 1;
#pragma unroll
        for (int q = 1; q < M - 1; ++q) {
            lam_p = add_fp64(lam_p, Llam[p[q]]);
            if (p[q] == p[q - 1]) {
                ++run;
                den *= double(run);
            } else {
                run = 1;
            }
        }
        const int m = p[M - 2];
        const double w_gt = -1.0 / den, w_eq = -1.0 / (den * double(run + 1));
        const float w_gt_f = float(w_gt), w_eq_f = float(w_eq);

        v4f rr[KTW], ri[KTW], rrl[KTW], ril[KTW];
#pragma unroll
        for (int kk = 0; kk < KTW; ++kk) rr[kk] = ri[kk] = rrl[kk] = ril[kk] = v4f{0, 0, 0, 0};

        // First product for this wave's 16-row tile of every 32-row chunk tc (skipped when
        // all its t < last(p)), each K-chunk of the rows split once.
        const int tc0 = m / 32;
        v4f sra[KC], sia[KC], srla[KC], sila[KC];
#pragma unroll
        for (int tc = 0; tc < KC; ++tc) sra[tc] = sia[tc] = srla[tc] = sila[tc] = v4f{0, 0, 0, 0};
        if (wave_on) {
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
                Split3 xr, xi;
                split_x(xv[kc], xr, xi);
                const Split3 xng = negx3(xi);
#pragma unroll
                for (int tc = 0; tc < KC; ++tc) {
                    const int tb = tc * 32 + 16 * half;
                    if (tc < tc0 || tb + 16 <= m) continue;
                    Split3 pr, pi;
                    phi_frags<NP>(Lphi, kc * 32, tb + c, g, pr, pi);
                    mm6s(pr, xr, sra[tc], srla[tc]);
                    mm6s(pi, xng, sra[tc], srla[tc]);
                    mm6s(pr, xi, sia[tc], sila[tc]);
                    mm6s(pi, xr, sia[tc], sila[tc]);
                }
            }
            if (itn < a.items) load_rows(itn);
        }
#pragma unroll
        for (int tc = 0; tc < KC; ++tc) {
            if (tc < tc0) continue;         // uniform: m is the workgroup's
            const int t0 = tc * 32, tb = t0 + 16 * half;
            const v4f sr = sra[tc], si = sia[tc], srl = srla[tc], sil = sila[tc];
            // Divisor and division (FP64 divisor) for the tile's rows t = tb + 4g + r.
            // exchange layout [buf][jt][half][r][lane]: lane-contiguous, no bank conflicts
            float2 *xo = Lx + ((buf * 4 + jt) * 2 + half) * 4 * 64 + lane;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int t = tb + 4 * g + r;
                float vr = 0.f, vi = 0.f;
                if (j_ok && t >= m && t < nn) {
                    // D in FP64 in the fixed summation order; the clamp and the division
                    // run in FP64 below the guard (|D| < tau, or near eps), else in FP32.
                    const double2 acc = add_fp64(lam_p, Llam[t]);
                    const double2 d = make_double2(acc.x - lam_j.x, acc.y - lam_j.y);
                    const float dx = float(d.x), dy = float(d.y);
                    const float dd = dx * dx + dy * dy;
                    const float w = (t == m) ? w_eq_f : w_gt_f;
                    const float sx = sr[r] + srl[r], sy = si[r] + sil[r];
                    if (dd < guard) {
                        const double2 dc = divisor_fp64(acc, lam_j, a.eps);
                        const double f = ((t == m) ? w_eq : w_gt) / (dc.x * dc.x + dc.y * dc.y);
                        vr = float((double(sx) * dc.x + double(sy) * dc.y) * f);
                        vi = float((double(sy) * dc.x - double(sx) * dc.y) * f);
                    } else {
                        float rc = __builtin_amdgcn_rcpf(dd);
                        rc = rc * (2.0f - dd * rc);          // one Newton step
                        const float f = w * rc;
                        vr = (sx * dx + sy * dy) * f;
                        vi = (sy * dx - sx * dy) * f;
                    }
                }
                xo[r * 64] = make_float2(vr, vi);
            }
            __syncthreads();
            // The reduction's A operand: K slots s < 4 from tile 0, s >= 4 from tile 1.
            const float2 *xin = Lx + (buf * 4 + jt) * 2 * 4 * 64 + lane;
            float hre[8], him[8];
#pragma unroll
            for (int s8 = 0; s8 < 8; ++s8) {
                const float2 v = xin[s8 * 64];          // (half, r) = (s8 / 4, s8 % 4)
                hre[s8] = v.x;
                him[s8] = v.y;
            }
            buf ^= 1;
            if (!wave_on) continue;
            const Split3 ar_ = split8(hre), ai_ = split8(him);
            const Split3 an_ = negx3(ai_);
#pragma unroll
            for (int kk = 0; kk < KTW; ++kk) {
                const int k = (half * KTW + kk) * 16 + c;
                const int z0 = int(zeta_frag_index(t0 + 4 * g, k, NP));
                auto ld = [&](int pl) { return *reinterpret_cast<const v8bf *>(Lz + pl * N2 + z0); };
                Split3 zr_, zi_;
                zr_.h = ld(0); zr_.m = ld(1); zr_.l = ld(2);
                zi_.h = ld(3); zi_.m = ld(4); zi_.l = ld(5);
                mm6s(ar_, zr_, rr[kk], rrl[kk]);
                mm6s(an_, zi_, rr[kk], rrl[kk]);
                mm6s(ar_, zi_, ri[kk], ril[kk]);
                mm6s(ai_, zr_, ri[kk], ril[kk]);
            }
        }
        if (!wave_on) continue;
        // P += zp * R in FP64, zp[k] = prod_i zeta[p_i][k] (FP32 product, one rounding per
        // item; the sum over items is kept in FP64).
#pragma unroll
        for (int kk = 0; kk < KTW; ++kk) {
            const int k = (half * KTW + kk) * 16 + c;
            float2 z = a.zeta32[p[0] * NP + k];
#pragma unroll
            for (int q = 1; q < M - 1; ++q) {
                const float2 w = a.zeta32[p[q] * NP + k];
                z = make_float2(z.x * w.x - z.y * w.y, z.x * w.y + z.y * w.x);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float vr = rr[kk][r] + rrl[kk][r], vi = ri[kk][r] + ril[kk][r];
                pacc_r[kk][r] += double(vr * z.x - vi * z.y);
                pacc_i[kk][r] += double(vr * z.y + vi * z.x);
            }
        }
    }
    if (!wave_on) return;
    double2 *dst = a.parts + int64_t(bp.x) * a.Jpad * a.n;
#pragma unroll
    for (int kk = 0; kk < KTW; ++kk) {
        const int64_t k = (half * KTW + kk) * 16 + c;
        if (k >= a.n) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t j = jw + 4 * g + r;
            dst[j * a.n + k] = make_double2(pacc_r[kk][r], pacc_i[kk][r]);
        }
    }
}

template <int NP, int M>
__global__ void __launch_bounds__(kThreads)
fused_bf3(Bf3Args a)
{
    fused_bf3_body<NP, M>(a, BlockPos{blockIdx.x, gridDim.x, int(blockIdx.y), int(blockIdx.z), 0});
}

// The same for several systems in one launch: workgroups [first[s], first[s+1]) of grid.x
// run system s with the arguments as[s].
template <int NP, int M>
__global__ void __launch_bounds__(kThreads)
fused_bf3_multi(const Bf3Args *__restrict__ as, const int32_t *__restrict__ first, int nsys)
{
    const BlockPos bp = system_block(first, nsys);
    fused_bf3_body<NP, M>(as[bp.sys], bp);
}

}  // namespace

bool bf3_small_supported(const npf_plan_s *p)
{
    return p->prec == NPF_BF16X3 && (p->npad == 32 || p->npad == 64) && p->N <= 4;
}

hipError_t launch_fused_bf3(const npf_plan_s *p, int M, int64_t j0, int64_t J, const double *lam,
                            char *ws, int64_t groups, hipStream_t s)
{
    const Bf3Args a = fused_args(p, M, j0, J, lam, ws);
    const dim3 grid{unsigned(groups), unsigned((p->Jpad + 63) / 64), 1u};
    const size_t shm = size_t(24 * p->npad * p->npad + 16 * p->npad + 32768);
#define NPF_FUSED_CASE(NP_, M_)                                                   \
    if (p->npad == NP_ && M == M_) {                                             \
        set_lds_limit(fused_bf3<NP_, M_>, int(shm));                              \
        hipLaunchKernelGGL((fused_bf3<NP_, M_>), grid, dim3(kThreads), shm, s, a); \
        return hipGetLastError();                                                 \
    }
    NPF_FUSED_CASE(32, 2) NPF_FUSED_CASE(32, 3) NPF_FUSED_CASE(32, 4)
    NPF_FUSED_CASE(64, 2) NPF_FUSED_CASE(64, 3) NPF_FUSED_CASE(64, 4)
#undef NPF_FUSED_CASE
    return hipErrorInvalidValue;
}

// Items taken at once by a workgroup of the t-range kernels: four waves of 16 modes share
// the block's 16-mode tiles, the remaining waves take further items.

hipError_t launch_fused_bf3_multi(int npad, int M, const MultiLaunch &m)
{
    const dim3 grid{unsigned(m.groups), unsigned(m.gy), 1u};
    const size_t shm = size_t(24 * npad * npad + 16 * npad + 32768);
    const Bf3Args *as = static_cast<const Bf3Args *>(m.args);
#define NPF_FUSED_MULTI(NP_, M_)                                                           \
    if (npad == NP_ && M == M_) {                                                         \
        set_lds_limit(fused_bf3_multi<NP_, M_>, int(shm));                                 \
        hipLaunchKernelGGL((fused_bf3_multi<NP_, M_>), grid, dim3(kThreads), shm, m.stream, \
                           as, m.first, m.nsys);                                           \
        return hipGetLastError();                                                          \
    }
    NPF_FUSED_MULTI(32, 2) NPF_FUSED_MULTI(32, 3) NPF_FUSED_MULTI(32, 4)
    NPF_FUSED_MULTI(64, 2) NPF_FUSED_MULTI(64, 3) NPF_FUSED_MULTI(64, 4)
#undef NPF_FUSED_MULTI
    return hipErrorInvalidValue;
}

}  // namespace npf
