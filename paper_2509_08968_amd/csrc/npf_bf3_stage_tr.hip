// Split-BF16 chain stage for systems of 65 to 256 states, and the stage dispatcher.
#include "npf_bf3.h"

namespace npf {

namespace {

// ------------------------------------------------------------------ one chain stage, n > 64
// Same arithmetic as stage_bf3; a workgroup owns a range of TT t-tiles (grid.z) and keeps
// only that slice of the Phi^T planes in LDS.  NW waves: WPI = NW / IPW waves per item (one
// 16-mode tile each) and IPW items per iteration (item slot = wave / WPI); with eight waves
// two waves share each SIMD, so that one issues while the other waits.  The gathered rows
// are loaded PD K-chunks ahead: the chunk PD places later in the sequence of (item, chunk)
// is loaded into a register slot as soon as that slot's chunk has been split.  Every lane
// loads every row of its chunks: rows a >= n read the row of a = 0, whose product with the
// zero rows of the Phi planes adds nothing, and a lane whose next item is absent reloads its
// current item -- so the loads carry no branches.
template <int NP, int SUF, int TT, int IPW, int NW>
__device__ __forceinline__ void stage_bf3_tr_body(const Bf3Args &a, const BlockPos bp)
{
    constexpr int KC = NP / 32, TW = TT * 16, AG = NP / 8;
    constexpr int PD = (NW == 8) ? (KC % 2 == 0 ? 2 : 1) : ((NP == 192) ? 3 : KC);
    static_assert(KC % PD == 0, "chunk slots must repeat at every item");
    constexpr int WPI = NW / IPW;
    extern __shared__ __align__(16) char lds[];
    // Per iteration, three buffers in rotation: iteration k's tables are read in iterations
    // k-1 and k and rewritten in iteration k+2 before that iteration's barrier, i.e. after
    // every wave has passed the barrier of iteration k+1.  sidx: gather rows of each item
    // slot; sbase: the item's input block and output row offsets; sm: last(p), or -1 for an
    // absent item.
    __shared__ int32_t sidx[3][IPW][NP];
    __shared__ int64_t sbase[3][IPW][2];
    __shared__ int32_t sm[3][IPW];
    __shared__ int64_t rowoff[TW];
    const int t_base = int(bp.z) * TW;
    {
        // Slice [t_base, t_base + TW) of the six planes [pl][a/8][t][a%8].
        const int4 *gsrc = reinterpret_cast<const int4 *>(a.phiE);
        int4 *ldst = reinterpret_cast<int4 *>(lds);
        for (int x = threadIdx.x; x < 6 * AG * TW; x += blockDim.x) {
            const int tl = x % TW, ag = (x / TW) % AG, pl = x / (TW * AG);
            const int t = t_base + tl;
            ldst[x] = (t < NP) ? gsrc[(int64_t(pl) * AG + ag) * NP + t] : int4{0, 0, 0, 0};
        }
        for (int tl = threadIdx.x; tl < TW; tl += blockDim.x)
            rowoff[tl] = colex_term_c(t_base + tl, a.i) * a.U_suf * a.Jpad;
    }
    const __bf16 *Lphi = reinterpret_cast<const __bf16 *>(lds);
    constexpr int PL = NP * TW;      // elements per LDS plane

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int islot = wave / WPI;
    const int64_t jw = (int64_t(bp.y) * WPI + wave % WPI) * 16;
    const bool wave_on = jw < a.Jpad;
    const float2 *X = static_cast<const float2 *>(a.X) + jw + c;
    const uint32_t jp = uint32_t(a.Jpad);
    const int nn = int(a.n);
    const int64_t istride = int64_t(bp.gx) * IPW;
    // Items are prefix-major and prefixes in colex order, i.e. by their last element first:
    // the items with some t >= last(p) in this slice are the first nitems, those whose prefix
    // has its last element below t_base + TW (binom(L + i - 2, i - 1) prefixes, L that bound).
    const int64_t nitems = [&] {
        if (a.i < 2) return a.items;
        const int64_t L = (t_base + TW < nn) ? t_base + TW : nn;
        const int64_t np = colex_term_c(L, a.i - 1);
        return np * a.U_suf < a.items ? np * a.U_suf : a.items;
    }();

    // Tables of the items ib .. ib + IPW - 1 into buffer buf.
    auto build = [&](int64_t ib, int buf) {
        for (int xq = threadIdx.x; xq < IPW * NP; xq += blockDim.x) {
            const int q = xq / NP;
            const int x = xq - q * NP;
            const int64_t itq = ib + q;
            if (itq >= nitems) {
                if (x == 0) sm[buf][q] = -1;
                continue;
            }
            const int64_t rp = itq / a.U_suf, rs = itq - rp * a.U_suf;
            if (x == 0) {
                sbase[buf][q][0] = rp * a.U_in * a.Jpad;
                sbase[buf][q][1] = (rp * a.U_suf + rs) * a.Jpad;
                sm[buf][q] = (a.i > 1) ? int(tuple_at(a.ptab[rp], a.i - 2)) : 0;
            }
            const uint64_t pk = a.stab[rs];
            const int32_t xe = (x < nn) ? x : 0;
            int64_t r = 0;
            int qq = 0;
#pragma unroll
            for (int l = 0; l < SUF; ++l) {
                const int32_t sl = tuple_at(pk, l);
                if (sl <= xe) {
                    r += colex_term_c(sl, l + 1);
                    ++qq;
                } else {
                    r += colex_term_c(sl, l + 2);
                }
            }
            sidx[buf][q][x] = int32_t(r + colex_term_c(xe, qq + 1));
        }
    };
    // Whether this workgroup's t-range has any t >= last(p) (never for an absent item).
    auto active = [&](int m) { return m >= 0 && t_base + TW > m; };
    auto load_chunk = [&](const float2 *src, const int32_t *rows, int kc, float2 (&dst)[8]) {
#pragma unroll
        for (int q = 0; q < 8; ++q)
            dst[q] = src[uint64_t(uint32_t(rows[kc * 32 + 8 * g + q])) * jp];
    };

    // ib: the workgroup's first item of the iteration (uniform); it = ib + islot.
    int64_t ib = int64_t(bp.x) * IPW;
    int buf = 0;
    float2 ring[PD][8];       // slot kc % PD: chunk kc of the current item, then kc + PD
    if (ib < nitems) build(ib, 0);
    else if (threadIdx.x < IPW) sm[0][threadIdx.x] = -1;
    __syncthreads();          // also orders the LDS slice of Phi
    if (wave_on && active(sm[0][islot])) {
#pragma unroll
        for (int kc = 0; kc < PD; ++kc) load_chunk(X + sbase[0][islot][0], sidx[0][islot], kc, ring[kc]);
    }
    for (; ib < nitems; ib += istride, buf = (buf == 2) ? 0 : buf + 1) {
        const int64_t ibn = ib + istride;
        const int nbuf = (buf == 2) ? 0 : buf + 1;
        if (ibn < nitems) build(ibn, nbuf);
        else if (threadIdx.x < IPW) sm[nbuf][threadIdx.x] = -1;
        __syncthreads();
        const int m = sm[buf][islot];
        if (!wave_on || m < 0) continue;
        const bool next_on = active(sm[nbuf][islot]);
        const float2 *src = X + sbase[buf][islot][0];
        const int32_t *rows = sidx[buf][islot];
        // The next item's rows, or the current ones again when there is none.
        const float2 *src_n = next_on ? X + sbase[nbuf][islot][0] : src;
        const int32_t *rows_n = next_on ? sidx[nbuf][islot] : rows;
        if (!active(m)) {
            if (next_on) {
#pragma unroll
                for (int kc = 0; kc < PD; ++kc) load_chunk(src_n, rows_n, kc, ring[kc]);
            }
            continue;
        }
        const int tt0 = (m > t_base) ? (m - t_base) / 16 : 0;
        v4f sr[TT], si[TT], srl[TT], sil[TT];
        // Straight-line tile loops for each first active tile (no branches between MFMAs).
        auto sweep = [&](auto first) {
            constexpr int T0 = decltype(first)::value;
#pragma unroll
            for (int tt = 0; tt < TT; ++tt) sr[tt] = si[tt] = srl[tt] = sil[tt] = v4f{0, 0, 0, 0};
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
                Split3 xr, xi;
                split_x(ring[kc % PD], xr, xi);
                if (kc + PD < KC) load_chunk(src, rows, kc + PD, ring[kc % PD]);
                else load_chunk(src_n, rows_n, kc + PD - KC, ring[kc % PD]);
                const Split3 xng = negx3(xi);
#pragma unroll
                for (int tt = T0; tt < TT; ++tt) {
                    const int pidx = ((kc * 4 + g) * TW + tt * 16 + c) * 8;
                    Split3 pr, pi;
                    pr.h = *reinterpret_cast<const v8bf *>(Lphi + 0 * PL + pidx);
                    pr.m = *reinterpret_cast<const v8bf *>(Lphi + 1 * PL + pidx);
                    pr.l = *reinterpret_cast<const v8bf *>(Lphi + 2 * PL + pidx);
                    pi.h = *reinterpret_cast<const v8bf *>(Lphi + 3 * PL + pidx);
                    pi.m = *reinterpret_cast<const v8bf *>(Lphi + 4 * PL + pidx);
                    pi.l = *reinterpret_cast<const v8bf *>(Lphi + 5 * PL + pidx);
                    mm6s(pr, xr, sr[tt], srl[tt]);
                    mm6s(pi, xng, sr[tt], srl[tt]);
                    mm6s(pr, xi, si[tt], sil[tt]);
                    mm6s(pi, xr, si[tt], sil[tt]);
                }
            }
        };
        switch (tt0) {
        case 0: sweep(std::integral_constant<int, 0>{}); break;
        case 1: if constexpr (TT > 1) sweep(std::integral_constant<int, (TT > 1 ? 1 : 0)>{}); break;
        case 2: if constexpr (TT > 2) sweep(std::integral_constant<int, (TT > 2 ? 2 : 0)>{}); break;
        default: if constexpr (TT > 3) sweep(std::integral_constant<int, (TT > 3 ? 3 : 0)>{}); break;
        }
        float2 *dst = static_cast<float2 *>(a.out) + sbase[buf][islot][1] + jw + c;
#pragma unroll
        for (int tt = 0; tt < TT; ++tt) {
            if (tt < tt0) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int tl = tt * 16 + 4 * g + r;
                const int t = t_base + tl;
                if (t < m || t >= nn) continue;
                dst[rowoff[tl]] = make_float2(sr[tt][r] + srl[tt][r], si[tt][r] + sil[tt][r]);
            }
        }
    }
}

template <int NP, int SUF, int TT, int IPW, int NW>
__global__ void __launch_bounds__(NW * 64)
stage_bf3_tr(Bf3Args a)
{
    stage_bf3_tr_body<NP, SUF, TT, IPW, NW>(
        a, BlockPos{xcd_block(blockIdx.x, gridDim.x), gridDim.x, int(blockIdx.y), int(blockIdx.z), 0});
}

// The same for several systems in one launch: workgroups [first[s], first[s+1]) of grid.x
// run system s with the arguments as[s].
template <int NP, int SUF, int TT, int IPW>
__global__ void __launch_bounds__(512)
stage_bf3_tr_multi(const Bf3Args *__restrict__ as, const int32_t *__restrict__ first, int nsys)
{
    const BlockPos bp = system_block(first, nsys);
    stage_bf3_tr_body<NP, SUF, TT, IPW, 8>(as[bp.sys], bp);
}

// ------------------------------------------------------------------ one chain stage, n > 64,
// slices walked inside the workgroup.  The same arithmetic as stage_bf3_tr_body, with the
// loops swapped: a workgroup takes a batch of IPW items and runs it through every t-slice of
// Phi^T in turn (the slice in LDS is reloaded between slices) before the next batch, so the
// rows an item gathers for one slice are gathered again for the next while they are still in
// the L2 cache, instead of once per slice across the whole launch.  The rows do not depend on
// the slice: while a slice's last K-chunks compute, the first chunks of the same item are
// loaded for the next slice (of the next batch's item after the last slice, where every item
// has work since its t range ends at n - 1 >= last(p)).  Slices below the batch's smallest
// last(p) are skipped; an item skips the slices below its own.
template <int NP, int SUF, int TT, int IPW, int NW>
__global__ void __launch_bounds__(NW * 64)
stage_bf3_sl(Bf3Args a)
{
    constexpr int KC = NP / 32, TW = TT * 16, AG = NP / 8;
    constexpr int NZ = (NP + TW - 1) / TW;
    constexpr int PD = (KC % 2 == 0) ? 2 : 1;
    static_assert(KC % PD == 0, "chunk slots must repeat at every item");
    constexpr int WPI = NW / IPW;
    constexpr int PL = NP * TW;                  // elements per LDS plane of a slice
    constexpr int NV = 6 * AG * TW;              // 16-byte vectors per slice
    constexpr int LPT = (NV + NW * 64 - 1) / (NW * 64);
    extern __shared__ __align__(16) char lds[];
    // Tables of the current batch and the next (built at the top of the current batch, after
    // a barrier that ends every wave's use of that buffer).
    __shared__ int32_t sidx[2][IPW][NP];
    __shared__ int64_t sbase[2][IPW][2];
    __shared__ int32_t sm[2][IPW];
    __shared__ int64_t rowoff[TW];
    const __bf16 *Lphi = reinterpret_cast<const __bf16 *>(lds);

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int islot = wave / WPI;
    const int64_t jw = (int64_t(blockIdx.y) * WPI + wave % WPI) * 16;
    const bool wave_on = jw < a.Jpad;
    const float2 *X = static_cast<const float2 *>(a.X) + jw + c;
    const uint32_t jp = uint32_t(a.Jpad);
    const int nn = int(a.n);
    const int64_t istride = int64_t(gridDim.x) * IPW;

    auto build = [&](int64_t ib, int buf) {
        for (int xq = threadIdx.x; xq < IPW * NP; xq += blockDim.x) {
            const int q = xq / NP;
            const int x = xq - q * NP;
            const int64_t itq = ib + q;
            if (itq >= a.items) {
                if (x == 0) sm[buf][q] = -1;
                continue;
            }
            const int64_t rp = itq / a.U_suf, rs = itq - rp * a.U_suf;
            if (x == 0) {
                sbase[buf][q][0] = rp * a.U_in * a.Jpad;
                sbase[buf][q][1] = (rp * a.U_suf + rs) * a.Jpad;
                sm[buf][q] = (a.i > 1) ? int(tuple_at(a.ptab[rp], a.i - 2)) : 0;
            }
            const uint64_t pk = a.stab[rs];
            const int32_t xe = (x < nn) ? x : 0;
            int64_t r = 0;
            int qq = 0;
#pragma unroll
            for (int l = 0; l < SUF; ++l) {
                const int32_t sl = tuple_at(pk, l);
                if (sl <= xe) {
                    r += colex_term_c(sl, l + 1);
                    ++qq;
                } else {
                    r += colex_term_c(sl, l + 2);
                }
            }
            sidx[buf][q][x] = int32_t(r + colex_term_c(xe, qq + 1));
        }
    };
    // Slice z of the six planes [pl][a/8][t][a%8] into LDS: a thread issues eight loads before
    // their stores.
    auto load_slice = [&](int z) {
        const int t_base = z * TW;
        const int4 *gsrc = reinterpret_cast<const int4 *>(a.phiE);
        int4 *ldst = reinterpret_cast<int4 *>(lds);
#pragma unroll
        for (int u0 = 0; u0 < LPT; u0 += 8) {
            int4 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int x = threadIdx.x + (u0 + u) * NW * 64;
                const int tl = x % TW, ag = (x / TW) % AG, pl = x / (TW * AG);
                const int t = t_base + tl;
                v[u] = (u0 + u < LPT && x < NV && t < NP) ? gsrc[(int64_t(pl) * AG + ag) * NP + t]
                                                          : int4{0, 0, 0, 0};
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int x = threadIdx.x + (u0 + u) * NW * 64;
                if (u0 + u < LPT && x < NV) ldst[x] = v[u];
            }
        }
        for (int tl = threadIdx.x; tl < TW; tl += blockDim.x)
            rowoff[tl] = colex_term_c(t_base + tl, a.i) * a.U_suf * a.Jpad;
    };
    auto load_chunk = [&](const float2 *src, const int32_t *rows, int kc, float2 (&dst)[8]) {
#pragma unroll
        for (int q = 0; q < 8; ++q)
            dst[q] = src[uint64_t(uint32_t(rows[kc * 32 + 8 * g + q])) * jp];
    };

    float2 ring[PD][8];       // slot kc % PD: chunk kc of the current unit, then kc + PD
    int64_t ib = int64_t(xcd_block(blockIdx.x, gridDim.x)) * IPW;
    if (ib < a.items) build(ib, 0);
    else if (threadIdx.x < IPW) sm[0][threadIdx.x] = -1;
    __syncthreads();
    if (wave_on && sm[0][islot] >= 0) {
#pragma unroll
        for (int kc = 0; kc < PD; ++kc) load_chunk(X + sbase[0][islot][0], sidx[0][islot], kc, ring[kc]);
    }
    int cur_z = -1;
    for (int buf = 0; ib < a.items; ib += istride, buf ^= 1) {
        const int64_t ibn = ib + istride;
        __syncthreads();                  // every wave is done with the other buffer
        if (ibn < a.items) build(ibn, buf ^ 1);
        else if (threadIdx.x < IPW) sm[buf ^ 1][threadIdx.x] = -1;
        __syncthreads();
        const int m = sm[buf][islot];
        const bool on = wave_on && m >= 0;
        const bool next_on = wave_on && sm[buf ^ 1][islot] >= 0;
        const float2 *src = X + (on ? sbase[buf][islot][0] : 0);
        const int32_t *rows = sidx[buf][islot];
        const float2 *src_n = X + (next_on ? sbase[buf ^ 1][islot][0] : 0);
        const int32_t *rows_n = sidx[buf ^ 1][islot];
        const int64_t obase = on ? sbase[buf][islot][1] : 0;
        for (int z = sm[buf][0] / TW; z < NZ; ++z) {
            if (z != cur_z) {
                __syncthreads();          // every wave is done with the previous slice
                load_slice(z);
                __syncthreads();
                cur_z = z;
            }
            const bool last = z == NZ - 1;
            const int t_base = z * TW;
            if (!on) {
                if (last && next_on) {
#pragma unroll
                    for (int kc = 0; kc < PD; ++kc) load_chunk(src_n, rows_n, kc, ring[kc]);
                }
                continue;
            }
            if (t_base + TW <= m) continue;      // the ring keeps this item's first chunks
            // The unit after this one: the same item at the next slice, or the next batch's.
            const float2 *nsrc = last ? src_n : src;
            const int32_t *nrows = last ? rows_n : rows;
            const bool nval = last ? next_on : true;
            const int tt0 = (m > t_base) ? (m - t_base) / 16 : 0;
            v4f sr[TT], si[TT], srl[TT], sil[TT];
            auto sweep = [&](auto first) {
                constexpr int T0 = decltype(first)::value;
#pragma unroll
                for (int tt = 0; tt < TT; ++tt) sr[tt] = si[tt] = srl[tt] = sil[tt] = v4f{0, 0, 0, 0};
#pragma unroll
                for (int kc = 0; kc < KC; ++kc) {
                    Split3 xr, xi;
                    split_x(ring[kc % PD], xr, xi);
                    if (kc + PD < KC) load_chunk(src, rows, kc + PD, ring[kc % PD]);
                    else if (nval) load_chunk(nsrc, nrows, kc + PD - KC, ring[kc % PD]);
                    // Issue the gathers before this chunk's products: left to itself the
                    // scheduler sinks them below the MFMAs, and the next chunk then waits
                    // for memory with no work in between.  (Not at 160 and 256 states, where
                    // the pinned order needs more registers than a wave has.)
                    if constexpr (NP != 160 && NP != 256) __builtin_amdgcn_sched_barrier(0);
                    const Split3 xng = negx3(xi);
#pragma unroll
                    for (int tt = T0; tt < TT; ++tt) {
                        if (t_base + tt * 16 >= nn) continue;   // a tile of padding rows only
                        const int pidx = ((kc * 4 + g) * TW + tt * 16 + c) * 8;
                        Split3 pr, pi;
                        pr.h = *reinterpret_cast<const v8bf *>(Lphi + 0 * PL + pidx);
                        pr.m = *reinterpret_cast<const v8bf *>(Lphi + 1 * PL + pidx);
                        pr.l = *reinterpret_cast<const v8bf *>(Lphi + 2 * PL + pidx);
                        pi.h = *reinterpret_cast<const v8bf *>(Lphi + 3 * PL + pidx);
                        pi.m = *reinterpret_cast<const v8bf *>(Lphi + 4 * PL + pidx);
                        pi.l = *reinterpret_cast<const v8bf *>(Lphi + 5 * PL + pidx);
                        mm6s(pr, xr, sr[tt], srl[tt]);
                        mm6s(pi, xng, sr[tt], srl[tt]);
                        mm6s(pr, xi, si[tt], sil[tt]);
                        mm6s(pi, xr, si[tt], sil[tt]);
                    }
                }
            };
            switch (tt0) {
            case 0: sweep(std::integral_constant<int, 0>{}); break;
            case 1: if constexpr (TT > 1) sweep(std::integral_constant<int, (TT > 1 ? 1 : 0)>{}); break;
            case 2: if constexpr (TT > 2) sweep(std::integral_constant<int, (TT > 2 ? 2 : 0)>{}); break;
            default: if constexpr (TT > 3) sweep(std::integral_constant<int, (TT > 3 ? 3 : 0)>{}); break;
            }
            float2 *dst = static_cast<float2 *>(a.out) + obase + jw + c;
#pragma unroll
            for (int tt = 0; tt < TT; ++tt) {
                if (tt < tt0) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int tl = tt * 16 + 4 * g + r;
                    const int t = t_base + tl;
                    if (t < m || t >= nn) continue;
                    dst[rowoff[tl]] = make_float2(sr[tt][r] + srl[tt][r], si[tt][r] + sil[tt][r]);
                }
            }
        }
    }
}

}  // namespace

hipError_t launch_stage_bf3(const ChainArgs &ca, int i)
{
    const npf_plan_s &p = *ca.plan;
    if (p.npad <= 64) return launch_stage_bf3_small(ca, i);
    const Bf3Args a = stage_args(ca, i);
    const int suf = ca.M - i;
    constexpr int nw = 8;
    const int ipw = bf3_items_per_group(p.Jpad) * nw / 4;     // items per batch
    const int64_t jgroups = (p.Jpad / 16 * ipw + nw - 1) / nw;
    int64_t groups = 512 / jgroups;
    const int64_t need = (a.items + ipw - 1) / ipw;
    if (groups > need) groups = need;
    if (groups >= 64) groups -= groups % 8;       // whole XCD rounds (xcd_block)
    if (groups < 1) groups = 1;
#define NPF_STAGE_RS(NP_, S_, TT_, IPW_, NW_)                                               \
    if (p.npad == NP_ && suf == S_ && ipw == IPW_ && nw == NW_) {                           \
        const dim3 grid{unsigned(groups), unsigned(jgroups), 1u};                           \
        const size_t shm = size_t(12 * NP_ * TT_ * 16);                                     \
        set_lds_limit(stage_bf3_sl<NP_, S_, TT_, IPW_, NW_>, int(shm));                      \
        hipLaunchKernelGGL((stage_bf3_sl<NP_, S_, TT_, IPW_, NW_>), grid, dim3(NW_ * 64), shm, \
                           ca.stream, a);                                                    \
        return hipGetLastError();                                                            \
    }
#define NPF_STAGE_RS_SUF(NP_, TT_, IPW_, NW_) \
    NPF_STAGE_RS(NP_, 1, TT_, IPW_, NW_) NPF_STAGE_RS(NP_, 2, TT_, IPW_, NW_) NPF_STAGE_RS(NP_, 3, TT_, IPW_, NW_)
#define NPF_STAGE_RS_8(NP_, TT_) \
    NPF_STAGE_RS_SUF(NP_, TT_, 2, 8) NPF_STAGE_RS_SUF(NP_, TT_, 4, 8) NPF_STAGE_RS_SUF(NP_, TT_, 8, 8)
#define NPF_STAGE_RS_4(NP_, TT_) \
    NPF_STAGE_RS_SUF(NP_, TT_, 1, 4) NPF_STAGE_RS_SUF(NP_, TT_, 2, 4) NPF_STAGE_RS_SUF(NP_, TT_, 4, 4)
    // The widest slice that fits LDS beside the tables.
    NPF_STAGE_RS_8(96, 3) NPF_STAGE_RS_8(128, 2) NPF_STAGE_RS_8(160, 3)
    NPF_STAGE_RS_8(192, 2) NPF_STAGE_RS_8(224, 2) NPF_STAGE_RS_8(256, 2)
#undef NPF_STAGE_RS_4
#undef NPF_STAGE_RS_8
#undef NPF_STAGE_RS_SUF
#undef NPF_STAGE_RS
    return hipErrorInvalidValue;
}

// t-tiles per workgroup of the t-range stage kernel for a system of npad states (as in
// launch_stage_bf3).
int stage_bf3_tr_tiles(int64_t npad) { return npad == 128 ? 4 : (npad == 256 ? 2 : 3); }

hipError_t launch_stage_bf3_tr_multi(int npad, int suf, const MultiLaunch &m)
{
    const int tt = stage_bf3_tr_tiles(npad);
    const dim3 grid{unsigned(m.groups), unsigned(m.gy), unsigned((npad / 16 + tt - 1) / tt)};
    const size_t shm = size_t(12 * npad * tt * 16);
    const Bf3Args *as = static_cast<const Bf3Args *>(m.args);
    // Eight waves: two items of up to 64 modes per iteration.
#define NPF_STAGE_TR_MULTI(NP_, S_, TT_)                                                       \
    if (npad == NP_ && suf == S_) {                                                           \
        set_lds_limit(stage_bf3_tr_multi<NP_, S_, TT_, 2>, int(shm));                          \
        hipLaunchKernelGGL((stage_bf3_tr_multi<NP_, S_, TT_, 2>), grid, dim3(512), shm,        \
                           m.stream, as, m.first, m.nsys);                                     \
        return hipGetLastError();                                                              \
    }
#define NPF_STAGE_TR_MULTI_NP(NP_, TT_) \
    NPF_STAGE_TR_MULTI(NP_, 1, TT_) NPF_STAGE_TR_MULTI(NP_, 2, TT_) NPF_STAGE_TR_MULTI(NP_, 3, TT_)
    NPF_STAGE_TR_MULTI_NP(96, 3) NPF_STAGE_TR_MULTI_NP(128, 4) NPF_STAGE_TR_MULTI_NP(160, 3)
    NPF_STAGE_TR_MULTI_NP(192, 3) NPF_STAGE_TR_MULTI_NP(224, 3) NPF_STAGE_TR_MULTI_NP(256, 2)
#undef NPF_STAGE_TR_MULTI_NP
#undef NPF_STAGE_TR_MULTI
    return hipErrorInvalidValue;
}

}  // namespace npf
