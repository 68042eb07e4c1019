// Split-BF16 fused last stage for systems of 65 to 256 states.
#include "npf_bf3.h"

namespace npf {

namespace {

// ------------------------------------------------------------------ fused last stage, n > 64
// Same arithmetic as fused_bf3; a workgroup owns one 32-wide t-slice (grid.z) of every
// item: the slices of Phi^T and zeta live in LDS, the reduction runs over the slice's t
// only, and the partial P of each (item group, slice, item slot) is summed with the others
// in the fixed-order partial sums (P is linear in the sum over t).
//
// Eight waves; the wave pair (w, w + 4) shares one SIMD and one (item slot, 16-mode tile).
// With fewer than four 16-mode tiles in the block the four pairs take IPW = 4 / tiles items
// at once (item slot = pair / (4 / IPW)), each slot writing its own partial.  Wave half h
// computes the first product over its half of the K-chunks (h = 0: chunks [0, KCH), h = 1:
// the rest); half 1 writes its partial sums to LDS, half 0 adds them to its own (half 0 +
// half 1, a fixed order) and writes the sum back, so both halves hold the same first
// product and divisor quotients.  The reduction's k tiles are split between the halves
// (h = 0: [0, KH), h = 1: [KH, NKT)), so each wave keeps half of the FP64 accumulators.
// For NP > 128 the states k are further split in KS ranges over grid.y (the first product
// is recomputed per range) so that the accumulators fit in registers and the zeta slice in
// LDS.
template <int NP, int M, int IPW, int KS>
__device__ __forceinline__ void fused_bf3_tr_body(const Bf3Args &a, const BlockPos bp)
{
    constexpr int NKT = NP / 16 / KS, KC = NP / 32, AG = NP / 8, N2 = NP * NP;
    constexpr int KW = NKT * 16;     // states k of this workgroup's range
    constexpr int KH = (NKT + 1) / 2, KCH = (KC + 1) / 2;
    constexpr int WPI = 4 / IPW;     // wave pairs per item
    constexpr int PLP = NP * 32;     // elements per LDS plane of the Phi^T slice
    constexpr int PLZ = 32 * KW;     // elements per LDS plane of the zeta slice
    extern __shared__ __align__(16) char lds[];
    __bf16 *Lphi = reinterpret_cast<__bf16 *>(lds);
    __bf16 *Lz = reinterpret_cast<__bf16 *>(lds + 12 * PLP);
    double2 *Llam = reinterpret_cast<double2 *>(lds + 12 * PLP + 12 * PLZ);
    // Exchange of the first product: [pair][value][lane], 16 values per lane.
    float *Lx = reinterpret_cast<float *>(lds + 12 * PLP + 12 * PLZ + 16 * NP);
    const int slice = int(bp.z), t_base = slice * 32;
    const int kh = int(bp.y) % KS, jgrp = int(bp.y) / KS;
    const int k_base = kh * KW;
    {
        const int4 *gp = reinterpret_cast<const int4 *>(a.phiE);
        int4 *lp = reinterpret_cast<int4 *>(Lphi);
        for (int x = threadIdx.x; x < 6 * AG * 32; x += blockDim.x) {
            const int tl = x % 32, ag = (x / 32) % AG, pl = x / (32 * AG);
            lp[x] = gp[(int64_t(pl) * AG + ag) * NP + t_base + tl];
        }
        const int4 *gz = reinterpret_cast<const int4 *>(a.zetaE);
        int4 *lz = reinterpret_cast<int4 *>(Lz);
        for (int x = threadIdx.x; x < 6 * 4 * KW; x += blockDim.x) {
            const int kk = x % KW, gg = (x / KW) % 4, pl = x / (4 * KW);
            lz[x] = gz[int64_t(pl) * (N2 / 8) + (int64_t(slice) * 4 + gg) * NP + k_base + kk];
        }
        for (int t = threadIdx.x; t < NP; t += blockDim.x)
            Llam[t] = t < a.n ? a.lam[t] : make_double2(0.0, 0.0);
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int pair = wave & 3, half = wave >> 2;
    const int g = lane >> 4, c = lane & 15;
    const int islot = pair / WPI;
    const int64_t jw = (int64_t(jgrp) * WPI + pair % WPI) * 16;
    const bool wave_on = jw < a.Jpad && islot < IPW;
    const int64_t jl = jw + c;
    const bool j_ok = wave_on && jl < a.J;
    const double2 lam_j = j_ok ? a.lamj[a.j0 + jl] : make_double2(0.0, 0.0);
    const float guard = fmaxf(float(a.tau2), float(4.0 * a.eps * a.eps));
    const int nn = int(a.n), jp = int(a.Jpad);
    const int64_t istride = int64_t(bp.gx) * IPW;
    const int kc0 = half * KCH, kcn = half ? KC - KCH : KCH;   // this half's K-chunks
    const int kt0 = half * KH, ktn = half ? NKT - KH : KH;     // this half's k tiles
    float *xs = Lx + pair * 16 * 64 + lane;

    double pacc_r[KH][4], pacc_i[KH][4];
#pragma unroll
    for (int kt = 0; kt < KH; ++kt)
#pragma unroll
        for (int r = 0; r < 4; ++r) pacc_r[kt][r] = pacc_i[kt][r] = 0.0;

    const float2 *X = static_cast<const float2 *>(a.X);
    // Rows a >= n read row n - 1: the Phi planes are zero there.
    const int rowlim = (nn - 1) * jp;
    auto load_chunk = [&](int64_t it, int kc, float2 (&dst)[8]) {
        const float2 *Xp = X + it * a.n * a.Jpad + jw + c;
        const int o0 = (kc * 32 + 8 * g) * jp;
#pragma unroll
        for (int s = 0; s < 8; ++s) dst[s] = Xp[min(o0 + s * jp, rowlim)];
    };
    auto last_of = [&](uint64_t pk) { return int(tuple_at(pk, M - 2)); };
    auto active = [&](uint64_t pk) { return t_base + 32 > last_of(pk); };

    // The item loop is uniform over the workgroup (it holds two barriers).
    const int64_t ib0 = int64_t(bp.x) * IPW;
    int64_t it = ib0 + islot;
    // Prefixes are in colex order (by their last element first): those with some t >=
    // last(p) in this slice are the first binom(L + M - 3, M - 2), L = min(t_base + 32, n).
    const int64_t nitems = [&] {
        const int64_t L = (t_base + 32 < nn) ? t_base + 32 : nn;
        const int64_t np = colex_term_c(L, M - 1);
        return np < a.items ? np : a.items;
    }();
    uint64_t pk = (it < nitems) ? a.ptab[it] : 0;
    float2 cur[8];
    if (wave_on && it < nitems && active(pk)) load_chunk(it, kc0, cur);
    for (int64_t ib = ib0; ib < nitems; ib += istride, it += istride) {
        // An offset the compiler cannot see through: the slices' fragments are read from LDS
        // in every iteration rather than hoisted into registers for the whole loop.
        int lo = 0;
        asm volatile("" : "+s"(lo));
        const __bf16 *Lp = Lphi + lo, *Lq = Lz + lo;
        const int64_t itn = it + istride;
        const uint64_t pkn = (itn < nitems) ? a.ptab[itn] : 0;
        const bool next_on = wave_on && itn < nitems && active(pkn);
        const bool on = wave_on && it < nitems && active(pk);
        v4f sr[2], si[2], srl[2], sil[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) sr[u] = si[u] = srl[u] = sil[u] = v4f{0, 0, 0, 0};
        const int m = on ? last_of(pk) : 0;
        if (on) {
            // First product over this half's K-chunks.  The chunk after the current one (or
            // the next item's first) is loaded into cur as soon as cur has been split.
            auto gemm1 = [&](auto first) {
                constexpr int U0 = decltype(first)::value;
#pragma unroll 1
                for (int kc = kc0; kc < kc0 + kcn; ++kc) {
                    Split3 xr, xi;
                    split_x(cur, xr, xi);
                    if (kc + 1 < kc0 + kcn) load_chunk(it, kc + 1, cur);
                    else if (next_on) load_chunk(itn, kc0, cur);
                    const Split3 xng = negx3(xi);
#pragma unroll
                    for (int u = U0; u < 2; ++u) {
                        // A tile of padding rows only (not at 160 states, where the test
                        // costs spills).
                        if constexpr (NP != 160)
                            if (t_base + 16 * u >= nn) continue;
                        const int pidx = ((kc * 4 + g) * 32 + 16 * u + c) * 8;
                        Split3 pr, pi;
                        pr.h = *reinterpret_cast<const v8bf *>(Lp + 0 * PLP + pidx);
                        pr.m = *reinterpret_cast<const v8bf *>(Lp + 1 * PLP + pidx);
                        pr.l = *reinterpret_cast<const v8bf *>(Lp + 2 * PLP + pidx);
                        pi.h = *reinterpret_cast<const v8bf *>(Lp + 3 * PLP + pidx);
                        pi.m = *reinterpret_cast<const v8bf *>(Lp + 4 * PLP + pidx);
                        pi.l = *reinterpret_cast<const v8bf *>(Lp + 5 * PLP + pidx);
                        mm6s(pr, xr, sr[u], srl[u]);
                        mm6s(pi, xng, sr[u], srl[u]);
                        mm6s(pr, xi, si[u], sil[u]);
                        mm6s(pi, xr, si[u], sil[u]);
                    }
                }
            };
            if (t_base + 16 > m) gemm1(std::integral_constant<int, 0>{});
            else gemm1(std::integral_constant<int, 1>{});
        } else if (next_on) {
            load_chunk(itn, kc0, cur);
        }
        // Exchange: half 1's partial sums -> half 0 adds its own -> the sum back to half 1.
        float sx[8], sy[8];
#pragma unroll
        for (int s8 = 0; s8 < 8; ++s8) {
            const int u = s8 >> 2, r = s8 & 3;
            sx[s8] = sr[u][r] + srl[u][r];
            sy[s8] = si[u][r] + sil[u][r];
        }
        if (on && half == 1) {
#pragma unroll
            for (int s8 = 0; s8 < 8; ++s8) {
                xs[(2 * s8) * 64] = sx[s8];
                xs[(2 * s8 + 1) * 64] = sy[s8];
            }
        }
        __syncthreads();
        if (on && half == 0) {
#pragma unroll
            for (int s8 = 0; s8 < 8; ++s8) {
                sx[s8] = sx[s8] + xs[(2 * s8) * 64];
                sy[s8] = sy[s8] + xs[(2 * s8 + 1) * 64];
                xs[(2 * s8) * 64] = sx[s8];
                xs[(2 * s8 + 1) * 64] = sy[s8];
            }
        }
        __syncthreads();
        if (on && half == 1) {
#pragma unroll
            for (int s8 = 0; s8 < 8; ++s8) {
                sx[s8] = xs[(2 * s8) * 64];
                sy[s8] = xs[(2 * s8 + 1) * 64];
            }
        }
        if (on) {
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
            const double w_gt = -1.0 / den, w_eq = -1.0 / (den * double(run + 1));
            const float w_gt_f = float(w_gt), w_eq_f = float(w_eq);
            // zp[k] = prod_i zeta[p_i][k] (FP32) for this half's k tiles.
            float2 zp[KH];
#pragma unroll
            for (int q = 0; q < KH; ++q) {
                const int k = k_base + (kt0 + q) * 16 + c;
                float2 z = make_float2(0.f, 0.f);
                if (q < ktn) {
                    z = a.zeta32[p[0] * NP + k];
#pragma unroll
                    for (int l = 1; l < M - 1; ++l) {
                        const float2 w = a.zeta32[p[l] * NP + k];
                        z = make_float2(z.x * w.x - z.y * w.y, z.x * w.y + z.y * w.x);
                    }
                }
                zp[q] = z;
            }
            // Divisor (FP64) and division into the reduction's A operand.
            float hre[8], him[8];
#pragma unroll
            for (int s8 = 0; s8 < 8; ++s8) {
                const int u = s8 >> 2, r = s8 & 3;
                const int t = t_base + 16 * u + 4 * g + r;
                float vr = 0.f, vi = 0.f;
                if (j_ok && t >= m && t < nn) {
                    const double2 acc = add_fp64(lam_p, Llam[t]);
                    const double2 d = make_double2(acc.x - lam_j.x, acc.y - lam_j.y);
                    const float dx = float(d.x), dy = float(d.y);
                    const float dd = dx * dx + dy * dy;
                    const float w = (t == m) ? w_eq_f : w_gt_f;
                    const float ax = sx[s8], ay = sy[s8];
                    if (dd < guard) {
                        const double2 dc = divisor_fp64(acc, lam_j, a.eps);
                        const double f = ((t == m) ? w_eq : w_gt) / (dc.x * dc.x + dc.y * dc.y);
                        vr = float((double(ax) * dc.x + double(ay) * dc.y) * f);
                        vi = float((double(ay) * dc.x - double(ax) * dc.y) * f);
                    } else {
                        float rc = __builtin_amdgcn_rcpf(dd);
                        rc = rc * (2.0f - dd * rc);
                        const float f = w * rc;
                        vr = (ax * dx + ay * dy) * f;
                        vi = (ay * dx - ax * dy) * f;
                    }
                }
                hre[s8] = vr;
                him[s8] = vi;
            }
            const Split3 ar_ = split8(hre), ai_ = split8(him);
            const Split3 an_ = negx3(ai_);
            // Second product over the slice (K = 32 t) for this half's k tiles.
#pragma unroll
            for (int q = 0; q < KH; ++q) {
                if (q >= ktn) break;
                const int kt = kt0 + q;
                const int z0 = (g * KW + kt * 16 + c) * 8;
                Split3 zr_, zi_;
                zr_.h = *reinterpret_cast<const v8bf *>(Lq + 0 * PLZ + z0);
                zr_.m = *reinterpret_cast<const v8bf *>(Lq + 1 * PLZ + z0);
                zr_.l = *reinterpret_cast<const v8bf *>(Lq + 2 * PLZ + z0);
                zi_.h = *reinterpret_cast<const v8bf *>(Lq + 3 * PLZ + z0);
                zi_.m = *reinterpret_cast<const v8bf *>(Lq + 4 * PLZ + z0);
                zi_.l = *reinterpret_cast<const v8bf *>(Lq + 5 * PLZ + z0);
                v4f rr = v4f{0, 0, 0, 0}, ri = v4f{0, 0, 0, 0};
                v4f rrl = v4f{0, 0, 0, 0}, ril = v4f{0, 0, 0, 0};
                mm6s(ar_, zr_, rr, rrl);
                mm6s(an_, zi_, rr, rrl);
                mm6s(ar_, zi_, ri, ril);
                mm6s(ai_, zr_, ri, ril);
                const float2 z = zp[q];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float vr = rr[r] + rrl[r], vi = ri[r] + ril[r];
                    pacc_r[q][r] += double(vr * z.x - vi * z.y);
                    pacc_i[q][r] += double(vr * z.y + vi * z.x);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        pk = pkn;
    }
    if (!wave_on) return;
    double2 *dst = a.parts + ((int64_t(bp.z) * bp.gx + bp.x) * IPW + islot) *
                                 a.Jpad * a.n;
#pragma unroll
    for (int q = 0; q < KH; ++q) {
        if (q >= ktn) break;
        const int64_t k = k_base + (kt0 + q) * 16 + c;
        if (k >= a.n) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t j = jw + 4 * g + r;
            dst[j * a.n + k] = make_double2(pacc_r[q][r], pacc_i[q][r]);
        }
    }
}

template <int NP, int M, int IPW, int KS>
__global__ void __launch_bounds__(512)
fused_bf3_tr(Bf3Args a)
{
    fused_bf3_tr_body<NP, M, IPW, KS>(a, BlockPos{blockIdx.x, gridDim.x, int(blockIdx.y), int(blockIdx.z), 0});
}

// The same for several systems in one launch: workgroups [first[s], first[s+1]) of grid.x
// run system s with the arguments as[s].
template <int NP, int M, int IPW, int KS>
__global__ void __launch_bounds__(512)
fused_bf3_tr_multi(const Bf3Args *__restrict__ as, const int32_t *__restrict__ first, int nsys)
{
    const BlockPos bp = system_block(first, nsys);
    fused_bf3_tr_body<NP, M, IPW, KS>(as[bp.sys], bp);
}

}  // namespace

int bf3_items_per_group(int64_t Jpad)
{
    const int64_t tiles = Jpad / 16;
    return tiles >= 3 ? 1 : int(4 / tiles);
}

// Partial slots written by the fused split-BF16 kernel for n > 64 per workgroup along x:
// t-slices x item slots.
int64_t fused_bf3_tr_slices(const npf_plan_s *p, int64_t Jpad)
{
    return p->npad / 32 * bf3_items_per_group(Jpad);
}

hipError_t launch_fused_bf3_tr(const npf_plan_s *p, int M, int64_t j0, int64_t J,
                               const double *lam, char *ws, int64_t groups, hipStream_t s)
{
    const Bf3Args a = fused_args(p, M, j0, J, lam, ws);
    const int NP = int(p->npad);
    const int ipw = bf3_items_per_group(p->Jpad);
    const int ks = fused_bf3_tr_kranges(NP);
    const int64_t jgroups = (p->Jpad / 16 * ipw + 3) / 4;
    const dim3 grid{unsigned(groups), unsigned(jgroups * ks), unsigned(NP / 32)};
    // LDS: the Phi^T and zeta slices, the eigenvalues, and the exchange of the first product.
    const size_t shm = size_t(12 * NP * 32 + 12 * 32 * (NP / ks) + 16 * NP + 4 * 16 * 64 * 4);
#define NPF_FUSED_TR(NP_, M_, IPW_)                                                             \
    if (NP == NP_ && M == M_ && ipw == IPW_) {                                                 \
        constexpr int KS_ = NP_ > 224 ? 4 : (NP_ > 160 ? 2 : 1);                               \
        set_lds_limit(fused_bf3_tr<NP_, M_, IPW_, KS_>, int(shm));                             \
        hipLaunchKernelGGL((fused_bf3_tr<NP_, M_, IPW_, KS_>), grid, dim3(512), shm, s, a);    \
        return hipGetLastError();                                                               \
    }
#define NPF_FUSED_TR_NP(NP_)                                                           \
    NPF_FUSED_TR(NP_, 2, 1) NPF_FUSED_TR(NP_, 3, 1) NPF_FUSED_TR(NP_, 4, 1)            \
    NPF_FUSED_TR(NP_, 2, 2) NPF_FUSED_TR(NP_, 3, 2) NPF_FUSED_TR(NP_, 4, 2)            \
    NPF_FUSED_TR(NP_, 2, 4) NPF_FUSED_TR(NP_, 3, 4) NPF_FUSED_TR(NP_, 4, 4)
    NPF_FUSED_TR_NP(96) NPF_FUSED_TR_NP(128) NPF_FUSED_TR_NP(160) NPF_FUSED_TR_NP(192)
    NPF_FUSED_TR_NP(224) NPF_FUSED_TR_NP(256)
#undef NPF_FUSED_TR_NP
#undef NPF_FUSED_TR
    return hipErrorInvalidValue;
}

bool bf3_tr_fused_supported(const npf_plan_s *p)
{
    return p->prec == NPF_BF16X3 && p->npad >= 96 && p->npad <= 256 && p->N <= 4;
}

// State ranges of the reduction for a system of npad states.
int fused_bf3_tr_kranges(int64_t npad) { return npad > 224 ? 4 : (npad > 160 ? 2 : 1); }

hipError_t launch_fused_bf3_tr_multi(int npad, int M, const MultiLaunch &m)
{
    const int ks = fused_bf3_tr_kranges(npad);
    const dim3 grid{unsigned(m.groups), unsigned(m.gy * ks), unsigned(npad / 32)};
    const size_t shm = size_t(12 * npad * 32 + 12 * 32 * (npad / ks) + 16 * npad + 4 * 16 * 64 * 4);
    const Bf3Args *as = static_cast<const Bf3Args *>(m.args);
#define NPF_FUSED_TR_MULTI(NP_, M_)                                                          \
    if (npad == NP_ && M == M_) {                                                           \
        constexpr int KS_ = NP_ > 224 ? 4 : (NP_ > 160 ? 2 : 1);                             \
        set_lds_limit(fused_bf3_tr_multi<NP_, M_, 1, KS_>, int(shm));                         \
        hipLaunchKernelGGL((fused_bf3_tr_multi<NP_, M_, 1, KS_>), grid, dim3(512), shm,      \
                           m.stream, as, m.first, m.nsys);                                   \
        return hipGetLastError();                                                            \
    }
#define NPF_FUSED_TR_MULTI_NP(NP_) NPF_FUSED_TR_MULTI(NP_, 2) NPF_FUSED_TR_MULTI(NP_, 3) NPF_FUSED_TR_MULTI(NP_, 4)
    NPF_FUSED_TR_MULTI_NP(96) NPF_FUSED_TR_MULTI_NP(128) NPF_FUSED_TR_MULTI_NP(160)
    NPF_FUSED_TR_MULTI_NP(192) NPF_FUSED_TR_MULTI_NP(224) NPF_FUSED_TR_MULTI_NP(256)
#undef NPF_FUSED_TR_MULTI_NP
#undef NPF_FUSED_TR_MULTI
    return hipErrorInvalidValue;
}

}  // namespace npf
