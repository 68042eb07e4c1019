// Split-BF16 kernels for systems of up to 64 states: the same arithmetic as the generic
// stage and fused kernels, organised for latency.  Every operand that is shared by the
// workgroup (Phi and zeta in their three-term BF16 planes, zeta in FP32 for the
// Khatri-Rao factor, the eigenvalues) lives in LDS for the whole launch; the grid is a
// few workgroups per CU that sweep the items, and the right operand rows of the next item
// are loaded into registers while the current item computes.
#include <type_traits>

#include "npf_device.h"
#include "npf_internal.h"
#include "npf_mfma.h"

namespace npf {

namespace {

constexpr int kThreads = 256;

struct Bf3Args {
    const void *X;           // fused: T_{M-1} [U_{M-1}][n][Jpad]; stage: T_{i-1}
    void *out;               // stage: T_i
    const __bf16 *phiE;      // 6 planes [pl][a/8][t][a%8]
    const __bf16 *zetaE;     // 6 planes [pl][t/4][k][t%4]
    const float2 *zeta32;    // [npad][npad] delta Psi
    const double2 *lam;      // [n]
    const uint64_t *ptab;    // sorted prefixes (fused: length M-1; stage: length i-1)
    const uint64_t *stab;    // stage: sorted suffixes of length M-i
    double2 *parts;          // fused: [gridDim.x][Jpad][n]
    int64_t n, Jpad, J, j0, items, U_suf, U_in;
    int M, i;
    double eps, tau2;
};

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

// ------------------------------------------------------------------ fused last stage
template <int NP, int M>
__global__ void __launch_bounds__(kThreads)
fused_bf3(Bf3Args a)
{
    constexpr int NKT = NP / 16, KC = NP / 32, N2 = NP * NP;
    extern __shared__ __align__(16) char lds[];
    __bf16 *Lphi = reinterpret_cast<__bf16 *>(lds);
    __bf16 *Lz = reinterpret_cast<__bf16 *>(lds + 12 * N2);
    float2 *Lz32 = reinterpret_cast<float2 *>(lds + 24 * N2);
    double2 *Llam = reinterpret_cast<double2 *>(lds + 32 * N2);
    copy_to_lds<NP>(lds, a.phiE, 12 * N2);
    copy_to_lds<NP>(lds + 12 * N2, a.zetaE, 12 * N2);
    copy_to_lds<NP>(lds + 24 * N2, a.zeta32, 8 * N2);
    for (int t = threadIdx.x; t < NP; t += blockDim.x)
        Llam[t] = t < a.n ? a.lam[t] : make_double2(0.0, 0.0);
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int64_t jw = int64_t(blockIdx.y) * 64 + wave * 16;
    const bool wave_on = jw < a.Jpad;
    const int64_t jl = jw + c;
    const bool j_ok = wave_on && jl < a.J;
    const double2 lam_j = j_ok ? Llam[a.j0 + jl] : make_double2(0.0, 0.0);
    // Below this |D|^2 (FP32) the divisor is finished in FP64: the tau band, and a margin
    // around eps so that the clamp is decided in FP64 exactly as specified.
    const float guard = fmaxf(float(a.tau2), float(4.0 * a.eps * a.eps));

    double pacc_r[NKT][4], pacc_i[NKT][4];
#pragma unroll
    for (int kt = 0; kt < NKT; ++kt)
#pragma unroll
        for (int r = 0; r < 4; ++r) pacc_r[kt][r] = pacc_i[kt][r] = 0.0;

    const float2 *X = static_cast<const float2 *>(a.X);
    float2 xn[KC][8];
    auto load_x = [&](int64_t it) {
        const float2 *Xp = X + it * a.n * a.Jpad + jw + c;
        const int jp = int(a.Jpad), nn = int(a.n);
#pragma unroll
        for (int kc = 0; kc < KC; ++kc)
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int ar = kc * 32 + 8 * g + s;
                xn[kc][s] = ar < nn ? Xp[ar * jp] : make_float2(0.f, 0.f);
            }
    };
    int64_t it = blockIdx.x;
    uint64_t pk_next = 0;
    if (wave_on && it < a.items) {
        load_x(it);
        pk_next = a.ptab[it];
    }
    if (wave_on)
    for (; it < a.items; it += gridDim.x) {
        // Split this item's rows, then start loading the next item's into the same registers.
        Split3 xr[KC], xi[KC], xn_[KC];
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            split_x(xn[kc], xr[kc], xi[kc]);
            xn_[kc] = negx3(xi[kc]);
        }
        const uint64_t pk = pk_next;
        const int64_t itn = it + gridDim.x;
        if (itn < a.items) {
            load_x(itn);
            pk_next = a.ptab[itn];
        }
        // Item constants (M is a compile-time constant: the tuple lives in registers).
        int32_t p[M - 1];
#pragma unroll
        for (int q = 0; q < M - 1; ++q) p[q] = int32_t((pk >> (8 * q)) & 0xff);
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

        v4f rr[NKT], ri[NKT];
#pragma unroll
        for (int kt = 0; kt < NKT; ++kt) rr[kt] = ri[kt] = v4f{0, 0, 0, 0};

        for (int tc = m / 32; tc < KC; ++tc) {
            const int t0 = tc * 32;
            v4f sr[2], si[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) sr[u] = si[u] = v4f{0, 0, 0, 0};
#pragma unroll
            for (int kc = 0; kc < KC; ++kc)
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    Split3 pr, pi;
                    phi_frags<NP>(Lphi, kc * 32, t0 + 16 * u + c, g, pr, pi);
                    sr[u] = mm6(pr, xr[kc], sr[u]);
                    sr[u] = mm6(pi, xn_[kc], sr[u]);
                    si[u] = mm6(pr, xi[kc], si[u]);
                    si[u] = mm6(pi, xr[kc], si[u]);
                }
            // Divisor and division (FP64 divisor) into the A operand of the reduction.
            float hre[8], him[8];
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int u = s >> 2, r = s & 3;
                const int t = t0 + 16 * u + 4 * g + r;
                float vr = 0.f, vi = 0.f;
                if (j_ok && t >= m && t < a.n) {
                    // D in FP64 in the fixed summation order; the clamp and the division
                    // run in FP64 below the guard (|D| < tau, or near eps), else in FP32.
                    const double2 acc = add_fp64(lam_p, Llam[t]);
                    const double2 d = make_double2(acc.x - lam_j.x, acc.y - lam_j.y);
                    const float dx = float(d.x), dy = float(d.y);
                    const float dd = dx * dx + dy * dy;
                    const float w = (t == m) ? w_eq_f : w_gt_f;
                    const float sx = sr[u][r], sy = si[u][r];
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
                hre[s] = vr;
                him[s] = vi;
            }
            const Split3 ar_ = split8(hre), ai_ = split8(him);
            const Split3 an_ = negx3(ai_);
#pragma unroll
            for (int kt = 0; kt < NKT; ++kt) {
                const int k = kt * 16 + c;
                const int z0 = int(zeta_frag_index(t0 + 4 * g, k, NP));
                auto ld = [&](int pl) { return *reinterpret_cast<const v8bf *>(Lz + pl * N2 + z0); };
                Split3 zr_, zi_;
                zr_.h = ld(0); zr_.m = ld(1); zr_.l = ld(2);
                zi_.h = ld(3); zi_.m = ld(4); zi_.l = ld(5);
                rr[kt] = mm6(ar_, zr_, rr[kt]);
                rr[kt] = mm6(an_, zi_, rr[kt]);
                ri[kt] = mm6(ar_, zi_, ri[kt]);
                ri[kt] = mm6(ai_, zr_, ri[kt]);
            }
        }
        // P += zp * R in FP64, zp[k] = prod_i zeta[p_i][k].
#pragma unroll
        for (int kt = 0; kt < NKT; ++kt) {
            const int k = kt * 16 + c;
            float2 z = Lz32[p[0] * NP + k];
#pragma unroll
            for (int q = 1; q < M - 1; ++q) {
                const float2 w = Lz32[p[q] * NP + k];
                z = make_float2(z.x * w.x - z.y * w.y, z.x * w.y + z.y * w.x);
            }
            // The item's product zp * R is formed in FP32 (one rounding); the sum over
            // items is kept in FP64.
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float vr = rr[kt][r], vi = ri[kt][r];
                pacc_r[kt][r] += double(vr * z.x - vi * z.y);
                pacc_i[kt][r] += double(vr * z.y + vi * z.x);
            }
        }
    }
    if (!wave_on) return;
    double2 *dst = a.parts + int64_t(blockIdx.x) * a.Jpad * a.n;
#pragma unroll
    for (int kt = 0; kt < NKT; ++kt) {
        const int64_t k = kt * 16 + c;
        if (k >= a.n) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t j = jw + 4 * g + r;
            dst[j * a.n + k] = make_double2(pacc_r[kt][r], pacc_i[kt][r]);
        }
    }
}

// ------------------------------------------------------------------ fused last stage, n > 64
// Same arithmetic as fused_bf3; a workgroup owns one 32-wide t-slice (grid.z) of every
// item: the slices of Phi^T and zeta live in LDS, the reduction runs over the slice's t
// only, and the partial P of each (item group, slice) workgroup is summed with the others
// in the fixed-order partial sums (P is linear in the sum over t).
template <int NP, int M>
__global__ void __launch_bounds__(kThreads)
fused_bf3_tr(Bf3Args a)
{
    constexpr int NKT = NP / 16, KC = NP / 32, AG = NP / 8, N2 = NP * NP;
    constexpr int PLP = NP * 32;     // elements per LDS plane of the Phi^T slice
    constexpr int PLZ = 32 * NP;     // elements per LDS plane of the zeta slice
    extern __shared__ __align__(16) char lds[];
    __bf16 *Lphi = reinterpret_cast<__bf16 *>(lds);
    __bf16 *Lz = reinterpret_cast<__bf16 *>(lds + 12 * PLP);
    double2 *Llam = reinterpret_cast<double2 *>(lds + 12 * PLP + 12 * PLZ);
    const int slice = int(blockIdx.z), t_base = slice * 32;
    {
        const int4 *gp = reinterpret_cast<const int4 *>(a.phiE);
        int4 *lp = reinterpret_cast<int4 *>(Lphi);
        for (int x = threadIdx.x; x < 6 * AG * 32; x += blockDim.x) {
            const int tl = x % 32, ag = (x / 32) % AG, pl = x / (32 * AG);
            lp[x] = gp[(int64_t(pl) * AG + ag) * NP + t_base + tl];
        }
        // zeta planes are in fragment order: the 32-row chunk of this slice is contiguous.
        const int4 *gz = reinterpret_cast<const int4 *>(a.zetaE);
        int4 *lz = reinterpret_cast<int4 *>(Lz);
        for (int x = threadIdx.x; x < 6 * 4 * NP; x += blockDim.x) {
            const int within = x % (4 * NP), pl = x / (4 * NP);
            lz[x] = gz[int64_t(pl) * (N2 / 8) + int64_t(slice) * 4 * NP + within];
        }
        for (int t = threadIdx.x; t < NP; t += blockDim.x)
            Llam[t] = t < a.n ? a.lam[t] : make_double2(0.0, 0.0);
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int64_t jw = int64_t(blockIdx.y) * 64 + wave * 16;
    const bool wave_on = jw < a.Jpad;
    const int64_t jl = jw + c;
    const bool j_ok = wave_on && jl < a.J;
    const double2 lam_j = j_ok ? Llam[a.j0 + jl] : make_double2(0.0, 0.0);
    const float guard = fmaxf(float(a.tau2), float(4.0 * a.eps * a.eps));
    const int nn = int(a.n), jp = int(a.Jpad);

    double pacc_r[NKT][4], pacc_i[NKT][4];
#pragma unroll
    for (int kt = 0; kt < NKT; ++kt)
#pragma unroll
        for (int r = 0; r < 4; ++r) pacc_r[kt][r] = pacc_i[kt][r] = 0.0;

    const float2 *X = static_cast<const float2 *>(a.X);
    auto load_chunk = [&](int64_t it, int kc, float2 (&dst)[8]) {
        const float2 *Xp = X + it * a.n * a.Jpad + jw + c;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int ar = kc * 32 + 8 * g + s;
            dst[s] = ar < nn ? Xp[ar * jp] : make_float2(0.f, 0.f);
        }
    };
    auto last_of = [&](uint64_t pk) { return int((pk >> (8 * (M - 2))) & 0xff); };
    // The slice has work for an item when some t in it is >= last(p).
    auto active = [&](uint64_t pk) { return t_base + 32 > last_of(pk); };

    int64_t it = blockIdx.x;
    uint64_t pk = (it < a.items) ? a.ptab[it] : 0;
    float2 cur[8];
    if (wave_on && it < a.items && active(pk)) load_chunk(it, 0, cur);
    if (wave_on)
    for (; it < a.items; it += gridDim.x) {
        const int64_t itn = it + gridDim.x;
        const uint64_t pkn = (itn < a.items) ? a.ptab[itn] : 0;
        const bool next_on = itn < a.items && active(pkn);
        if (!active(pk)) {
            if (next_on) load_chunk(itn, 0, cur);
            pk = pkn;
            continue;
        }
        int32_t p[M - 1];
#pragma unroll
        for (int q = 0; q < M - 1; ++q) p[q] = int32_t((pk >> (8 * q)) & 0xff);
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
        // zp[k] = prod_i zeta[p_i][k] (FP32), loaded now and used after the products.
        float2 zp[NKT];
#pragma unroll
        for (int kt = 0; kt < NKT; ++kt) {
            const int k = kt * 16 + c;
            float2 z = a.zeta32[p[0] * NP + k];
#pragma unroll
            for (int q = 1; q < M - 1; ++q) {
                const float2 w = a.zeta32[p[q] * NP + k];
                z = make_float2(z.x * w.x - z.y * w.y, z.x * w.y + z.y * w.x);
            }
            zp[kt] = z;
        }

        // GEMM1 over the slice's two t-tiles, rows loaded one K-chunk ahead.
        v4f sr[2], si[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) sr[u] = si[u] = v4f{0, 0, 0, 0};
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            float2 nxt[8];
            if (kc + 1 < KC) load_chunk(it, kc + 1, nxt);
            else if (next_on) load_chunk(itn, 0, nxt);
            Split3 xr, xi;
            split_x(cur, xr, xi);
            const Split3 xng = negx3(xi);
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int pidx = ((kc * 4 + g) * 32 + 16 * u + c) * 8;
                Split3 pr, pi;
                pr.h = *reinterpret_cast<const v8bf *>(Lphi + 0 * PLP + pidx);
                pr.m = *reinterpret_cast<const v8bf *>(Lphi + 1 * PLP + pidx);
                pr.l = *reinterpret_cast<const v8bf *>(Lphi + 2 * PLP + pidx);
                pi.h = *reinterpret_cast<const v8bf *>(Lphi + 3 * PLP + pidx);
                pi.m = *reinterpret_cast<const v8bf *>(Lphi + 4 * PLP + pidx);
                pi.l = *reinterpret_cast<const v8bf *>(Lphi + 5 * PLP + pidx);
                sr[u] = mm6(pr, xr, sr[u]);
                sr[u] = mm6(pi, xng, sr[u]);
                si[u] = mm6(pr, xi, si[u]);
                si[u] = mm6(pi, xr, si[u]);
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) cur[q] = nxt[q];
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
                const float sx = sr[u][r], sy = si[u][r];
                if (dd < guard) {
                    const double2 dc = divisor_fp64(acc, lam_j, a.eps);
                    const double f = ((t == m) ? w_eq : w_gt) / (dc.x * dc.x + dc.y * dc.y);
                    vr = float((double(sx) * dc.x + double(sy) * dc.y) * f);
                    vi = float((double(sy) * dc.x - double(sx) * dc.y) * f);
                } else {
                    float rc = __builtin_amdgcn_rcpf(dd);
                    rc = rc * (2.0f - dd * rc);
                    const float f = w * rc;
                    vr = (sx * dx + sy * dy) * f;
                    vi = (sy * dx - sx * dy) * f;
                }
            }
            hre[s8] = vr;
            him[s8] = vi;
        }
        const Split3 ar_ = split8(hre), ai_ = split8(him);
        const Split3 an_ = negx3(ai_);
        // GEMM2 over the slice (K = 32 t) for every k tile, then P += zp * R in FP64.
#pragma unroll
        for (int kt = 0; kt < NKT; ++kt) {
            const int z0 = (g * NP + kt * 16 + c) * 8;
            Split3 zr_, zi_;
            zr_.h = *reinterpret_cast<const v8bf *>(Lz + 0 * PLZ + z0);
            zr_.m = *reinterpret_cast<const v8bf *>(Lz + 1 * PLZ + z0);
            zr_.l = *reinterpret_cast<const v8bf *>(Lz + 2 * PLZ + z0);
            zi_.h = *reinterpret_cast<const v8bf *>(Lz + 3 * PLZ + z0);
            zi_.m = *reinterpret_cast<const v8bf *>(Lz + 4 * PLZ + z0);
            zi_.l = *reinterpret_cast<const v8bf *>(Lz + 5 * PLZ + z0);
            v4f rr = v4f{0, 0, 0, 0}, ri = v4f{0, 0, 0, 0};
            rr = mm6(ar_, zr_, rr);
            rr = mm6(an_, zi_, rr);
            ri = mm6(ar_, zi_, ri);
            ri = mm6(ai_, zr_, ri);
            const float2 z = zp[kt];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float vr = rr[r], vi = ri[r];
                pacc_r[kt][r] += double(vr * z.x - vi * z.y);
                pacc_i[kt][r] += double(vr * z.y + vi * z.x);
            }
        }
        pk = pkn;
    }
    if (!wave_on) return;
    double2 *dst = a.parts + (int64_t(blockIdx.z) * gridDim.x + blockIdx.x) * a.Jpad * a.n;
#pragma unroll
    for (int kt = 0; kt < NKT; ++kt) {
        const int64_t k = kt * 16 + c;
        if (k >= a.n) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t j = jw + 4 * g + r;
            dst[j * a.n + k] = make_double2(pacc_r[kt][r], pacc_i[kt][r]);
        }
    }
}

// ------------------------------------------------------------------ one chain stage
template <int NP, int SUF>
__global__ void __launch_bounds__(kThreads)
stage_bf3(Bf3Args a)
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
    const int64_t jw = int64_t(blockIdx.y) * 64 + wave * 16;
    const bool wave_on = jw < a.Jpad;
    const float2 *X = static_cast<const float2 *>(a.X);

    auto build_idx = [&](int64_t it, int buf) {
        const int64_t rs = it % a.U_suf;
        const uint64_t pk = a.stab[rs];
        if (threadIdx.x < a.n) {
            // rank(sort({x} U s)) for the sorted suffix s (SUF entries, in registers).
            const int32_t x = int32_t(threadIdx.x);
            int64_t r = 0;
            int q = 0;
#pragma unroll
            for (int l = 0; l < SUF; ++l) {
                const int32_t sl = int32_t((pk >> (8 * l)) & 0xff);
                if (sl <= x) {
                    r += colex_term_c(sl, l + 1);
                    ++q;
                } else {
                    r += colex_term_c(sl, l + 2);
                }
            }
            sidx[buf][threadIdx.x] = int32_t(r + colex_term_c(x, q + 1));
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

    int64_t it = blockIdx.x;
    int buf = 0;
    if (it < a.items) build_idx(it, 0);
    __syncthreads();          // also orders the LDS copy of Phi
    if (it < a.items && wave_on) gather_x(it, 0);
    for (; it < a.items; it += gridDim.x, buf ^= 1) {
        Split3 xr[KC], xi[KC], xn_[KC];
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            split_x(xn[kc], xr[kc], xi[kc]);
            xn_[kc] = negx3(xi[kc]);
        }
        const int64_t itn = it + gridDim.x;
        if (itn < a.items) build_idx(itn, buf ^ 1);
        __syncthreads();
        if (itn < a.items && wave_on) gather_x(itn, buf ^ 1);
        if (!wave_on) continue;

        const int64_t rp = it / a.U_suf, rs = it % a.U_suf;
        int m = 0;
        if (a.i > 1) m = int((a.ptab[rp] >> (8 * (a.i - 2))) & 0xff);
        const int tt0 = m / 16;

        v4f sr[NTT], si[NTT];
#pragma unroll
        for (int tt = 0; tt < NTT; ++tt) sr[tt] = si[tt] = v4f{0, 0, 0, 0};
#pragma unroll
        for (int tt = 0; tt < NTT; ++tt) {
            if (tt < tt0) continue;
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
                Split3 pr, pi;
                phi_frags<NP>(Lphi, kc * 32, tt * 16 + c, g, pr, pi);
                sr[tt] = mm6(pr, xr[kc], sr[tt]);
                sr[tt] = mm6(pi, xn_[kc], sr[tt]);
                si[tt] = mm6(pr, xi[kc], si[tt]);
                si[tt] = mm6(pi, xr[kc], si[tt]);
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
                dst[rowoff[t]] = make_float2(sr[tt][r], si[tt][r]);
            }
        }
    }
}

// ------------------------------------------------------------------ one chain stage, n > 64
// Same arithmetic as stage_bf3; a workgroup owns a range of TT t-tiles (grid.z) and keeps
// only that slice of the Phi^T planes in LDS.  The gathered rows are loaded one K-chunk
// ahead (the last chunk of an item prefetches the first chunk of the next item).
template <int NP, int SUF, int TT>
__global__ void __launch_bounds__(kThreads)
stage_bf3_tr(Bf3Args a)
{
    constexpr int KC = NP / 32, TW = TT * 16, AG = NP / 8;
    extern __shared__ __align__(16) char lds[];
    // Gather tables, three buffers in rotation: item k's table is read in iterations k-1
    // (its first chunk) and k (the others) and rewritten in iteration k+2 before that
    // iteration's barrier, i.e. after every wave has passed the barrier of iteration k+1.
    __shared__ int32_t sidx[3][NP];
    __shared__ int64_t rowoff[TW];
    const int t_base = int(blockIdx.z) * TW;
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
    const int64_t jw = int64_t(blockIdx.y) * 64 + wave * 16;
    const bool wave_on = jw < a.Jpad;
    const float2 *X = static_cast<const float2 *>(a.X);
    const unsigned jp = unsigned(a.Jpad);
    const int nn = int(a.n);

    auto build_idx = [&](int64_t it, int buf) {
        const uint64_t pk = a.stab[it % a.U_suf];
        if (threadIdx.x < a.n) {
            const int32_t x = int32_t(threadIdx.x);
            int64_t r = 0;
            int q = 0;
#pragma unroll
            for (int l = 0; l < SUF; ++l) {
                const int32_t sl = int32_t((pk >> (8 * l)) & 0xff);
                if (sl <= x) {
                    r += colex_term_c(sl, l + 1);
                    ++q;
                } else {
                    r += colex_term_c(sl, l + 2);
                }
            }
            sidx[buf][threadIdx.x] = int32_t(r + colex_term_c(x, q + 1));
        }
    };
    // last(p) of an item, and whether this workgroup's t-range has any t >= last(p).
    auto item_m = [&](int64_t it) {
        return (a.i > 1) ? int((a.ptab[it / a.U_suf] >> (8 * (a.i - 2))) & 0xff) : 0;
    };
    auto active = [&](int m) { return t_base + TW > m; };
    auto load_chunk = [&](int64_t it, int buf, int kc, float2 (&dst)[8]) {
        const float2 *src = X + (it / a.U_suf) * a.U_in * a.Jpad + jw + c;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int ar = kc * 32 + 8 * g + q;
            dst[q] = ar < nn ? src[uint64_t(unsigned(sidx[buf][ar])) * jp] : make_float2(0.f, 0.f);
        }
    };

    int64_t it = blockIdx.x;
    int buf = 0;
    float2 cur[8];
    if (it < a.items) build_idx(it, 0);
    __syncthreads();          // also orders the LDS slice of Phi
    if (it < a.items && wave_on && active(item_m(it))) load_chunk(it, 0, 0, cur);
    for (; it < a.items; it += gridDim.x, buf = (buf == 2) ? 0 : buf + 1) {
        const int64_t itn = it + gridDim.x;
        const int nbuf = (buf == 2) ? 0 : buf + 1;
        if (itn < a.items) build_idx(itn, nbuf);
        __syncthreads();
        if (!wave_on) continue;
        const int m = item_m(it);
        const bool next_on = itn < a.items && active(item_m(itn));
        if (!active(m)) {
            if (next_on) load_chunk(itn, nbuf, 0, cur);
            continue;
        }
        const int tt0 = (m > t_base) ? (m - t_base) / 16 : 0;
        v4f sr[TT], si[TT];
        // Straight-line tile loops for each first active tile (no branches between MFMAs).
        auto sweep = [&](auto first) {
            constexpr int T0 = decltype(first)::value;
#pragma unroll
            for (int tt = 0; tt < TT; ++tt) sr[tt] = si[tt] = v4f{0, 0, 0, 0};
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
                float2 nxt[8];
                if (kc + 1 < KC) load_chunk(it, buf, kc + 1, nxt);
                else if (next_on) load_chunk(itn, nbuf, 0, nxt);
                Split3 xr, xi;
                split_x(cur, xr, xi);
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
                    sr[tt] = mm6(pr, xr, sr[tt]);
                    sr[tt] = mm6(pi, xng, sr[tt]);
                    si[tt] = mm6(pr, xi, si[tt]);
                    si[tt] = mm6(pi, xr, si[tt]);
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) cur[q] = nxt[q];
            }
        };
        switch (tt0) {
        case 0: sweep(std::integral_constant<int, 0>{}); break;
        case 1: if constexpr (TT > 1) sweep(std::integral_constant<int, (TT > 1 ? 1 : 0)>{}); break;
        case 2: if constexpr (TT > 2) sweep(std::integral_constant<int, (TT > 2 ? 2 : 0)>{}); break;
        default: if constexpr (TT > 3) sweep(std::integral_constant<int, (TT > 3 ? 3 : 0)>{}); break;
        }
        const int64_t rp = it / a.U_suf, rs = it % a.U_suf;
        float2 *dst = static_cast<float2 *>(a.out) + (rp * a.U_suf + rs) * a.Jpad + jw + c;
#pragma unroll
        for (int tt = 0; tt < TT; ++tt) {
            if (tt < tt0) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int tl = tt * 16 + 4 * g + r;
                const int t = t_base + tl;
                if (t < m || t >= nn) continue;
                dst[rowoff[tl]] = make_float2(sr[tt][r], si[tt][r]);
            }
        }
    }
}

template <typename K>
void set_lds_limit(K kernel, int bytes)
{
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

Bf3Args base_args(const npf_plan_s *p, char *ws, const double *lam)
{
    const int64_t N2 = p->npad * p->npad;
    char *base = ws + p->lay.phi;
    Bf3Args a{};
    a.phiE = reinterpret_cast<const __bf16 *>(base + 16 * N2);
    a.zetaE = reinterpret_cast<const __bf16 *>(base + 34 * N2);
    a.zeta32 = reinterpret_cast<const float2 *>(base + 50 * N2);
    a.lam = reinterpret_cast<const double2 *>(lam);
    a.n = p->n;
    a.Jpad = p->Jpad;
    a.eps = p->prob.eps;
    a.tau2 = p->prob.tau * p->prob.tau;
    return a;
}

}  // namespace

bool bf3_small_supported(const npf_plan_s *p)
{
    return p->prec == NPF_BF16X3 && (p->npad == 32 || p->npad == 64) && p->N <= 4;
}

hipError_t launch_fused_bf3(const npf_plan_s *p, int M, int64_t j0, int64_t J, const double *lam,
                            char *ws, int64_t groups, hipStream_t s)
{
    Bf3Args a = base_args(p, ws, lam);
    a.X = ws + p->lay.buf[(M - 1) % 2];
    a.ptab = reinterpret_cast<const uint64_t *>(ws + p->lay.ttab) + p->tt.off[M - 1];
    a.parts = reinterpret_cast<double2 *>(ws + p->lay.parts);
    a.J = J;
    a.j0 = j0;
    a.items = p->U[M - 1];
    a.M = M;
    const dim3 grid{unsigned(groups), unsigned((p->Jpad + 63) / 64), 1u};
    const size_t shm = size_t(32 * p->npad * p->npad + 16 * p->npad);
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

// Partial slots written by the fused split-BF16 kernel for n > 64: groups x slices.
int64_t fused_bf3_tr_slices(const npf_plan_s *p) { return p->npad / 32; }

hipError_t launch_fused_bf3_tr(const npf_plan_s *p, int M, int64_t j0, int64_t J,
                               const double *lam, char *ws, int64_t groups, hipStream_t s)
{
    Bf3Args a = base_args(p, ws, lam);
    a.X = ws + p->lay.buf[(M - 1) % 2];
    a.ptab = reinterpret_cast<const uint64_t *>(ws + p->lay.ttab) + p->tt.off[M - 1];
    a.parts = reinterpret_cast<double2 *>(ws + p->lay.parts);
    a.J = J;
    a.j0 = j0;
    a.items = p->U[M - 1];
    a.M = M;
    const int NP = int(p->npad);
    const dim3 grid{unsigned(groups), unsigned((p->Jpad + 63) / 64), unsigned(NP / 32)};
    const size_t shm = size_t(24 * NP * 32 + 16 * NP);
#define NPF_FUSED_TR(NP_, M_)                                                                 \
    if (NP == NP_ && M == M_) {                                                              \
        set_lds_limit(fused_bf3_tr<NP_, M_>, int(shm));                                       \
        hipLaunchKernelGGL((fused_bf3_tr<NP_, M_>), grid, dim3(kThreads), shm, s, a);         \
        return hipGetLastError();                                                             \
    }
    NPF_FUSED_TR(96, 2) NPF_FUSED_TR(96, 3) NPF_FUSED_TR(96, 4)
    NPF_FUSED_TR(128, 2) NPF_FUSED_TR(128, 3) NPF_FUSED_TR(128, 4)
#undef NPF_FUSED_TR
    return hipErrorInvalidValue;
}

bool bf3_tr_fused_supported(const npf_plan_s *p)
{
    return p->prec == NPF_BF16X3 && (p->npad == 96 || p->npad == 128) && p->N <= 4;
}

hipError_t launch_stage_bf3(const ChainArgs &ca, int i)
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
    const int64_t jgroups = (p.Jpad + 63) / 64;
    int64_t groups = 512 / jgroups;
    if (groups > a.items) groups = a.items;
    if (groups < 1) groups = 1;
    const int suf = M - i;
    if (p.npad <= 64) {
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
#define NPF_STAGE_TR(NP_, S_, TT_)                                                         \
    if (p.npad == NP_ && suf == S_) {                                                      \
        const dim3 grid{unsigned(groups), unsigned(jgroups), unsigned((NP_ / 16 + TT_ - 1) / TT_)}; \
        const size_t shm = size_t(12 * NP_ * TT_ * 16);                                    \
        set_lds_limit(stage_bf3_tr<NP_, S_, TT_>, int(shm));                                \
        hipLaunchKernelGGL((stage_bf3_tr<NP_, S_, TT_>), grid, dim3(kThreads), shm, ca.stream, a); \
        return hipGetLastError();                                                           \
    }
    NPF_STAGE_TR(96, 1, 3) NPF_STAGE_TR(96, 2, 3) NPF_STAGE_TR(96, 3, 3)
    NPF_STAGE_TR(128, 1, 4) NPF_STAGE_TR(128, 2, 4) NPF_STAGE_TR(128, 3, 4)
    NPF_STAGE_TR(160, 1, 2) NPF_STAGE_TR(160, 2, 2) NPF_STAGE_TR(160, 3, 2)
    NPF_STAGE_TR(192, 1, 2) NPF_STAGE_TR(192, 2, 2) NPF_STAGE_TR(192, 3, 2)
    NPF_STAGE_TR(224, 1, 2) NPF_STAGE_TR(224, 2, 2) NPF_STAGE_TR(224, 3, 2)
    NPF_STAGE_TR(256, 1, 2) NPF_STAGE_TR(256, 2, 2) NPF_STAGE_TR(256, 3, 2)
#undef NPF_STAGE_TR
    return hipErrorInvalidValue;
}

bool bf3_stage_supported(const npf_plan_s *p)
{
    return p->prec == NPF_BF16X3 && p->N <= 4;
}

}  // namespace npf
