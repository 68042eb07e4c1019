// One stage of the lower-index chain on MFMA (Alg. 2 steps 2-3, one mode product each):
//   T_i[rank(p U t)][rs][j] = sum_a T_{i-1}[rp][rank(sort(a U s))][j] Phi[a][t],  t >= last(p)
// for every sorted mode prefix p (length i-1, rank rp) and sorted state suffix s (length
// M-i, rank rs).  Per (p, s) item this is a [t x a] x [a x j] complex product whose right
// operand rows are gathered from the symmetric storage of T_{i-1}; the gather table
// rank(sort(a U s)) is built once per item in LDS (double-buffered, one barrier per item).
// Wave w of a workgroup owns 16 modes and sweeps NTT t tiles of the item: the t tiles are
// dealt to grid.z in groups of NTT (at most four, so that the accumulators leave registers
// for two waves per SIMD), and a row is gathered once per group.  Phi stays in LDS when it
// fits.  The gathered row of the next K-step is loaded while the current one's products run.
#include "npf_device.h"
#include "npf_internal.h"
#include "npf_mfma.h"

namespace npf {

namespace {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kMaxN = 512;          // states supported by the MFMA kernels
constexpr int64_t kResidentBytes = 128 * 1024;

struct StageArgs {
    const void *in;        // T_{i-1}: [U_{i-1}][U_in][Jpad]
    void *out;             // T_i:     [U_i][U_suf][Jpad]
    const void *phiE;      // staged Phi (engine layout)
    const uint64_t *ptab;  // sorted (i-1)-tuples (unused when i == 1)
    const uint64_t *stab;  // sorted (M-i)-tuples (unused when i == M)
    int64_t n, npad, Jpad, U_suf, U_in, items;
    int M, i;
};

template <Eng E> constexpr int64_t phi_bytes(int64_t npad)
{
    return (E == Eng::F64 ? 16 : (E == Eng::F32 ? 8 : 12)) * npad * npad;
}

template <Eng E, int NTT, bool RES>
__global__ void __launch_bounds__(kThreads, 2)
stage_mfma(StageArgs a)
{
    using T = EngT<E>;
    using acc_t = typename T::acc;
    using real = typename T::real;
    using cplx = typename T::cplx;
    extern __shared__ __align__(16) char lds[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int64_t jw = int64_t(blockIdx.y) * 64 + wave * 16;
    const bool wave_on = jw < a.Jpad;
    const int ntt = int((a.n + 15) / 16);           // t tiles holding some t < n
    const int tz0 = int(blockIdx.z) * NTT;          // first t tile of this group
    const int64_t N2 = a.npad * a.npad;

    __shared__ int32_t sidx[2][kMaxN];

    const char *phiB = static_cast<const char *>(a.phiE);
    if constexpr (RES) {
        const int4 *gp = reinterpret_cast<const int4 *>(a.phiE);
        int4 *lp = reinterpret_cast<int4 *>(lds);
        for (int64_t x = threadIdx.x; x < phi_bytes<E>(a.npad) / 16; x += blockDim.x) lp[x] = gp[x];
        phiB = lds;      // the barrier of the first item orders these writes
    }

    const int sufl = a.M - a.i;       // suffix length
    int parity = 0;
    for (int64_t it = blockIdx.x; it < a.items; it += gridDim.x, parity ^= 1) {
        const int64_t rp = it / a.U_suf, rs = it % a.U_suf;
        int32_t p[NPF_MAX_ORDER], s[NPF_MAX_ORDER];
        if (a.i > 1) unpack_tuple(a.ptab[rp], a.i - 1, p);
        if (sufl > 0) unpack_tuple(a.stab[rs], sufl, s);
        const int m = (a.i > 1) ? p[a.i - 2] : 0;
        {
            InsertRank ir;
            ir.init(s, sufl);
            for (int x = threadIdx.x; x < a.n; x += blockDim.x)
                sidx[parity][x] = int32_t(ir.rank(int32_t(x)));
        }
        __syncthreads();
        const int tt0 = m / 16;
        if (!wave_on || tz0 + NTT <= tt0) continue;        // no t >= m in this group
        const int32_t *idx = sidx[parity];
        const cplx *src = static_cast<const cplx *>(a.in) + rp * a.U_in * a.Jpad + jw + c;

        acc_t sr[NTT], si[NTT];
#pragma unroll
        for (int tt = 0; tt < NTT; ++tt) sr[tt] = si[tt] = acc_t{0, 0, 0, 0};

        if constexpr (E != Eng::BF3) {
            const cplx *Ph = reinterpret_cast<const cplx *>(phiB);
            auto gather = [&](int64_t ar) {
                return ar < a.n ? src[int64_t(idx[ar]) * a.Jpad] : cplx{0, 0};
            };
            cplx xn = gather(g);
            for (int64_t a0 = 0; a0 < a.npad; a0 += 4) {
                const int64_t ar = a0 + g;
                const cplx x = xn;
                if (a0 + 4 < a.npad) xn = gather(ar + 4);
#pragma unroll
                for (int tt = 0; tt < NTT; ++tt) {
                    const int tg = tz0 + tt;
                    if (tg < tt0 || tg >= ntt) continue;
                    const cplx ph = Ph[ar * a.npad + tg * 16 + c];
                    sr[tt] = mfma(ph.x, x.x, sr[tt]);
                    sr[tt] = mfma(real(-ph.y), x.y, sr[tt]);
                    si[tt] = mfma(ph.x, x.y, si[tt]);
                    si[tt] = mfma(ph.y, x.x, si[tt]);
                }
            }
        } else {
            const __bf16 *Ph = reinterpret_cast<const __bf16 *>(phiB);
            for (int64_t a0 = 0; a0 < a.npad; a0 += 32) {
                Split3 xr, xi;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int64_t ar = a0 + 8 * g + q;
                    float2 x = make_float2(0.f, 0.f);
                    if (ar < a.n) x = src[int64_t(idx[ar]) * a.Jpad];
                    __bf16 h, mm, l;
                    split3(x.x, h, mm, l);
                    xr.h[q] = h; xr.m[q] = mm; xr.l[q] = l;
                    split3(x.y, h, mm, l);
                    xi.h[q] = h; xi.m[q] = mm; xi.l[q] = l;
                }
#pragma unroll
                for (int tt = 0; tt < NTT; ++tt) {
                    const int tg = tz0 + tt;
                    if (tg < tt0 || tg >= ntt) continue;
                    const int64_t pidx = ((a0 / 8 + g) * a.npad + tg * 16 + c) * 8;
                    Split3 pr, pi;
                    pr.h = *reinterpret_cast<const v8bf *>(Ph + 0 * N2 + pidx);
                    pr.m = *reinterpret_cast<const v8bf *>(Ph + 1 * N2 + pidx);
                    pr.l = *reinterpret_cast<const v8bf *>(Ph + 2 * N2 + pidx);
                    pi.h = *reinterpret_cast<const v8bf *>(Ph + 3 * N2 + pidx);
                    pi.m = *reinterpret_cast<const v8bf *>(Ph + 4 * N2 + pidx);
                    pi.l = *reinterpret_cast<const v8bf *>(Ph + 5 * N2 + pidx);
                    const Split3 pn = neg3(pi);
                    sr[tt] = mm6(pr, xr, sr[tt]);
                    sr[tt] = mm6(pn, xi, sr[tt]);
                    si[tt] = mm6(pr, xi, si[tt]);
                    si[tt] = mm6(pi, xr, si[tt]);
                }
            }
        }
        // Store T_i rows (p U t, s) for t >= m; rank(p U t) = rp + binom(t + i - 1, i).
        cplx *dst = static_cast<cplx *>(a.out) + rs * a.Jpad + jw + c;
#pragma unroll
        for (int tt = 0; tt < NTT; ++tt) {
            const int tg = tz0 + tt;
            if (tg < tt0 || tg >= ntt) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t t = int64_t(tg) * 16 + out_row<E>(r, g);
                if (t < m || t >= a.n) continue;
                const int64_t row = rp + colex_term_c(t, a.i);
                dst[row * a.U_suf * a.Jpad] = cplx{real(sr[tt][r]), real(si[tt][r])};
            }
        }
    }
}

template <Eng E, int NTT, bool RES>
void launch_one(const dim3 &grid, const StageArgs &sa, hipStream_t s)
{
    const size_t shm = RES ? size_t(phi_bytes<E>(sa.npad)) : 0;
    if (RES) {
        static bool attr = false;
        if (!attr) {
            (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&stage_mfma<E, NTT, RES>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, int(kResidentBytes));
            attr = true;
        }
    }
    hipLaunchKernelGGL((stage_mfma<E, NTT, RES>), grid, dim3(kThreads), shm, s, sa);
}

template <Eng E>
hipError_t launch_stage_eng(const StageArgs &sa, int ntt, int64_t jgroups, hipStream_t s)
{
    // t tiles per workgroup: two or four (tiles past the last one holding some t < n are
    // skipped), more in groups of four over grid.z.
    const int tg = ntt <= 2 ? 2 : 4;
    const int64_t zg = (ntt + tg - 1) / tg;
    int64_t groups = 1024 / (jgroups * zg);
    if (groups > sa.items) groups = sa.items;
    if (groups < 1) groups = 1;
    const dim3 grid{unsigned(groups), unsigned(jgroups), unsigned(zg)};
    const bool res = phi_bytes<E>(sa.npad) <= kResidentBytes;
    if (tg == 2) {
        if (res) launch_one<E, 2, true>(grid, sa, s);
        else launch_one<E, 2, false>(grid, sa, s);
    } else if (tg == 4) {
        if (res) launch_one<E, 4, true>(grid, sa, s);
        else launch_one<E, 4, false>(grid, sa, s);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

bool stage_mfma_supported(const npf_plan_s *p) { return p->n <= kMaxN; }

hipError_t launch_stage_mfma(const ChainArgs &ca, int i)
{
    const npf_plan_s &p = *ca.plan;
    if (bf3_stage_supported(&p)) return launch_stage_bf3(ca, i);
    const int M = ca.M;
    const uint64_t *tt = reinterpret_cast<const uint64_t *>(ca.ws + p.lay.ttab);
    StageArgs sa;
    sa.in = ca.ws + p.lay.buf[(i - 1) % 2];
    sa.out = ca.ws + p.lay.buf[i % 2];
    sa.phiE = ca.ws + p.lay.phi + 16 * p.npad * p.npad;
    sa.ptab = tt + p.tt.off[i - 1 > 0 ? i - 1 : 1];
    sa.stab = tt + p.tt.off[M - i > 0 ? M - i : 1];
    sa.n = p.n;
    sa.npad = p.npad;
    sa.Jpad = p.Jpad;
    sa.U_suf = p.U[M - i];
    sa.U_in = p.U[M - i + 1];
    sa.items = p.U[i - 1] * p.U[M - i];
    sa.M = M;
    sa.i = i;
    const int ntt = int((p.n + 15) / 16);
    const int64_t jgroups = (p.Jpad + 63) / 64;
    switch (p.prec) {
    case NPF_FP64: return launch_stage_eng<Eng::F64>(sa, ntt, jgroups, ca.stream);
    case NPF_FP32: return launch_stage_eng<Eng::F32>(sa, ntt, jgroups, ca.stream);
    default: return launch_stage_eng<Eng::BF3>(sa, ntt, jgroups, ca.stream);
    }
}

}  // namespace npf
