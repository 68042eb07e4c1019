// Fused last stage of the chain on MFMA: for every sorted mode prefix p of length M-1,
//   S[t][j]  = sum_a Phi[a][t] X_p[a][j]                       (last mode product, t >= last(p))
//   h'[j][t] = S[t][j] W(p,t) / D(j, p U t)                     (divisor in FP64, Alg. 2 steps 5-11)
//   P[j][k] += zp[k] sum_t h'[j][t] zeta[t][k]                  (Alg. 2 steps 12-19)
// with X_p = T_{M-1}[p] (all upper-index and M-1 lower-index contractions done),
// zeta = delta Psi, zp[k] = prod_i zeta[p_i][k], W(p,t) = -1/prod_v c_v! over the value
// counts of the sorted tuple p U t (the orderings of the tuple times 1/M!), and
// D = (lam_{p_1} + .. + lam_{p_{M-1}} + lam_t) - lam_j, |D| < eps -> eps.
// h' never leaves registers: the accumulator layout of the first product is re-used as
// the A operand of the second.  Each workgroup accumulates its items in FP64 and writes
// one partial; two small kernels sum the partials in a fixed order (deterministic).
#include "npf_device.h"
#include "npf_internal.h"
#include "npf_mfma.h"

namespace npf {

namespace {

constexpr int kWaves = 4;               // one 16-mode j-tile per wave
constexpr int kThreads = 64 * kWaves;
constexpr int64_t kResidentBytes = 128 * 1024;   // LDS budget for resident operands

// ------------------------------------------------------------------ operand staging
// zeta64[t][k] = delta Psi[t][k] (FP64, zero padded to npad).  Engine copies:
//   F64: phi[a][t], zeta[t][k] as double2;  F32: the same as float2;
//   BF3: phi as 6 BF16 planes (re h/m/l, im h/m/l) in layout [pl][a/8][t][a%8],
//        zeta as 6 planes (re h/m/l, im h/m/l) in the fragment order of zeta_frag_index.
// Also the tables of sorted tuples of length 1..N-1 (9 bits per entry), in colex order.
// With selected modes, also the Psi rows and (when lam is given) the eigenvalues of the
// computed modes: msel[c*n + k] = Psi[row[c], k] and msel[nc*n + c] = lam[row[c]].
// With zadd (the sum over orders of P_M, [mode][state]) the reduction's factor becomes the
// corrected zeta* = delta Psi + zadd of eq. (9) (the interaction factors of eq. (8)).
__global__ void __launch_bounds__(256)
prepare(const double2 *__restrict__ Phi, const double2 *__restrict__ Psi, double delta, int64_t n,
        int64_t npad, int eng, double2 *__restrict__ zeta64, void *__restrict__ phiE,
        void *__restrict__ zetaE, float2 *__restrict__ zeta32, uint64_t *__restrict__ ttab,
        TupleTables tt, const double2 *__restrict__ lam, double2 *__restrict__ msel, int64_t nc,
        ModeMap mm, const double2 *__restrict__ zadd)
{
    const int64_t N2 = npad * npad;
    const int64_t nsel = msel ? nc * (n + 1) : 0;
    const int64_t total = N2 + tt.total + nsel;
    for (int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < total;
         x += int64_t(gridDim.x) * blockDim.x) {
        if (x >= N2 + tt.total) {
            const int64_t y = x - N2 - tt.total;
            if (y < nc * n) {
                const int64_t c = y / n, k = y - c * n;
                msel[y] = Psi[int64_t(mm.row[c]) * n + k];
            } else if (lam) {
                msel[y] = lam[mm.row[y - nc * n]];
            }
            continue;
        }
        if (x >= N2) {
            int64_t y = x - N2;
            int m = 1;
            while (m < tt.maxlen && y >= tt.count[m]) {
                y -= tt.count[m];
                ++m;
            }
            int32_t t[NPF_MAX_ORDER];
            colex_unrank(y, m, n, t);
            uint64_t pk = 0;
            for (int i = 0; i < m; ++i) pk |= tuple_entry(t[i], i);
            ttab[tt.off[m] + y] = pk;
            continue;
        }
        const int64_t r = x / npad, c = x % npad;   // r = a or t, c = t or k
        const bool in = r < n && c < n;
        const double2 ph = in ? Phi[r * n + c] : make_double2(0.0, 0.0);
        double2 ze = in ? Psi[r * n + c] : make_double2(0.0, 0.0);
        ze = make_double2(delta * ze.x, delta * ze.y);
        if (zadd && in) ze = add_fp64(ze, zadd[r * n + c]);   // zeta* = zeta + sum_M P_M (eq. (9))
        zeta64[x] = ze;
        zeta32[x] = make_float2(float(ze.x), float(ze.y));
        if (eng == int(Eng::F64)) {
            static_cast<double2 *>(phiE)[x] = ph;
            static_cast<double2 *>(zetaE)[x] = ze;
        } else if (eng == int(Eng::F32)) {
            static_cast<float2 *>(phiE)[x] = make_float2(float(ph.x), float(ph.y));
            static_cast<float2 *>(zetaE)[x] = make_float2(float(ze.x), float(ze.y));
        } else {
            __bf16 *P = static_cast<__bf16 *>(phiE);
            const int64_t pidx = ((r / 8) * npad + c) * 8 + (r % 8);    // a = r, t = c
            __bf16 h, m, l;
            split3(float(ph.x), h, m, l);
            P[0 * N2 + pidx] = h; P[1 * N2 + pidx] = m; P[2 * N2 + pidx] = l;
            split3(float(ph.y), h, m, l);
            P[3 * N2 + pidx] = h; P[4 * N2 + pidx] = m; P[5 * N2 + pidx] = l;
            __bf16 *Z = static_cast<__bf16 *>(zetaE);
            const int64_t zidx = zeta_frag_index(r, c, npad);            // t = r, k = c
            split3(float(ze.x), h, m, l);
            Z[0 * N2 + zidx] = h; Z[1 * N2 + zidx] = m; Z[2 * N2 + zidx] = l;
            split3(float(ze.y), h, m, l);
            Z[3 * N2 + zidx] = h; Z[4 * N2 + zidx] = m; Z[5 * N2 + zidx] = l;
        }
    }
}

// h' = S W / D for one element; FP64 divisor, FP64 or FP32 division (the FP32 engine, whose
// products are accumulated in FP64, divides in FP64 too: one rounding of h' to FP32).
template <Eng E, typename Sv>
__device__ __forceinline__ void scaled_quotient(Sv sr, Sv si, double2 d, double w, double tau2,
                                                typename EngT<E>::real &hr, typename EngT<E>::real &hi)
{
    const double den = d.x * d.x + d.y * d.y;
    if constexpr (E == Eng::F64 || E == Eng::F32) {
        const double f = w / den;
        hr = (double(sr) * d.x + double(si) * d.y) * f;
        hi = (double(si) * d.x - double(sr) * d.y) * f;
    } else {
        if (den < tau2) {
            const double f = w / den;
            hr = float((double(sr) * d.x + double(si) * d.y) * f);
            hi = float((double(si) * d.x - double(sr) * d.y) * f);
        } else {
            const float dx = float(d.x), dy = float(d.y);
            const float f = float(w) / (dx * dx + dy * dy);
            hr = (sr * dx + si * dy) * f;
            hi = (si * dx - sr * dy) * f;
        }
    }
}

struct FusedArgs {
    const void *X;           // T_{M-1}: [U_{M-1}][n][Jpad] complex
    const void *phiE;        // staged Phi (engine layout)
    const void *zetaE;       // staged zeta (engine layout)
    const double2 *zeta64;   // [npad][npad] delta Psi
    const double2 *lam;      // [n]
    const double2 *lamj;     // eigenvalues of the computed modes (mode j0 + jl)
    const uint64_t *ptab;    // sorted (M-1)-tuples, packed
    double2 *parts;          // [gridDim.x][Jpad][n]
    int64_t n, npad, Jpad, J, j0, items;
    int M;
    double eps, tau2;
};

template <Eng E> constexpr int64_t resident_bytes(int64_t npad)
{
    return (E == Eng::F64 ? 32 : (E == Eng::F32 ? 16 : 24)) * npad * npad;
}

// ------------------------------------------------------------------ the fused kernel
// grid: x = item groups (grid-stride over prefixes), y = 64-mode j-groups, z = k-groups of
// NKTW 16-state tiles.  Block: 4 waves, wave w owns modes jg*64 + 16w .. +15.  With RES the
// Phi and zeta operands are copied to LDS once and every fragment is read from there.
template <Eng E, int NKTW, bool RES>
__global__ void __launch_bounds__(kThreads)
fused_last(FusedArgs a)
{
    using T = EngT<E>;
    using acc_t = typename T::acc;
    using real = typename T::real;
    using cplx = typename T::cplx;
    extern __shared__ __align__(16) char lds[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int64_t jw = int64_t(blockIdx.y) * 64 + wave * 16;     // wave's first mode (block-local)
    const bool wave_on = jw < a.Jpad;
    const int64_t jl = jw + c;                                   // this lane's mode (block-local)
    const bool j_ok = wave_on && jl < a.J;
    const double2 lam_j = j_ok ? a.lamj[a.j0 + jl] : make_double2(0.0, 0.0);
    const int kt0 = blockIdx.z * NKTW;
    const int nkt = int(a.npad / 16);
    constexpr int TC = T::TC;
    const int64_t N2 = a.npad * a.npad;

    // Operand bases: LDS copies (RES) or the staged global copies.
    const char *phiB = static_cast<const char *>(a.phiE);
    const char *zetaB = static_cast<const char *>(a.zetaE);
    if constexpr (RES) {
        const int64_t half = resident_bytes<E>(a.npad) / 2;
        const int4 *gp = reinterpret_cast<const int4 *>(a.phiE);
        const int4 *gz = reinterpret_cast<const int4 *>(a.zetaE);
        int4 *lp = reinterpret_cast<int4 *>(lds);
        int4 *lz = reinterpret_cast<int4 *>(lds + half);
        for (int64_t x = threadIdx.x; x < half / 16; x += blockDim.x) {
            lp[x] = gp[x];
            lz[x] = gz[x];
        }
        __syncthreads();
        phiB = lds;
        zetaB = lds + half;
    }

    // FP64 accumulators of this lane: P[jw + out_row(r,g)][(kt0+kt)*16 + c].
    double pacc_r[NKTW][4], pacc_i[NKTW][4];
#pragma unroll
    for (int kt = 0; kt < NKTW; ++kt)
#pragma unroll
        for (int r = 0; r < 4; ++r) pacc_r[kt][r] = pacc_i[kt][r] = 0.0;

    if (wave_on)
    for (int64_t it = blockIdx.x; it < a.items; it += gridDim.x) {
        // ---------------- item constants (uniform): p, last(p), lam sum, weights.
        int32_t p[NPF_MAX_ORDER];
        unpack_tuple(a.ptab[it], a.M - 1, p);
        double2 lam_p = a.lam[p[0]];
        double den = 1.0;
        int run = 1;
        for (int i = 1; i < a.M - 1; ++i) {
            lam_p = add_fp64(lam_p, a.lam[p[i]]);
            if (p[i] == p[i - 1]) {
                ++run;
                den *= double(run);
            } else {
                run = 1;
            }
        }
        const int m = p[a.M - 2];
        const double w_gt = -1.0 / den, w_eq = -1.0 / (den * double(run + 1));
        const cplx *Xp = static_cast<const cplx *>(a.X) + it * a.n * a.Jpad;

        // zp[k] for this lane's k columns (FP64).
        double zr[NKTW], zi[NKTW];
#pragma unroll
        for (int kt = 0; kt < NKTW; ++kt) {
            const int64_t k = int64_t(kt0 + kt) * 16 + c;
            double2 z = make_double2(1.0, 0.0);
            if ((kt0 + kt) < nkt)
                for (int i = 0; i < a.M - 1; ++i) z = cmul(z, a.zeta64[int64_t(p[i]) * a.npad + k]);
            zr[kt] = z.x;
            zi[kt] = z.y;
        }

        // Per-item GEMM2 accumulators (FP32 engines; the FP64 engine accumulates directly).
        acc_t rr[NKTW], ri[NKTW];
#pragma unroll
        for (int kt = 0; kt < NKTW; ++kt) rr[kt] = ri[kt] = acc_t{0, 0, 0, 0};

        for (int64_t t0 = (m / TC) * TC; t0 < a.n; t0 += TC) {     // chunks holding some t < n
            // ---------------- GEMM1: S^T[t][j] over a, tiles of 16 t.
            constexpr int NT1 = (E == Eng::BF3) ? 2 : 1;
            acc_t sr[NT1], si[NT1];
#pragma unroll
            for (int u = 0; u < NT1; ++u) sr[u] = si[u] = acc_t{0, 0, 0, 0};
            if constexpr (E != Eng::BF3) {
                const cplx *Ph = reinterpret_cast<const cplx *>(phiB);
                for (int64_t a0 = 0; a0 < a.npad; a0 += 4) {
                    const int64_t ar = a0 + g;
                    const cplx ph = Ph[ar * a.npad + t0 + c];
                    cplx x;
                    if (ar < a.n) x = Xp[ar * a.Jpad + jw + c];
                    else x = cplx{0, 0};
                    sr[0] = mfma(ph.x, x.x, sr[0]);
                    sr[0] = mfma(real(-ph.y), x.y, sr[0]);
                    si[0] = mfma(ph.x, x.y, si[0]);
                    si[0] = mfma(ph.y, x.x, si[0]);
                }
            } else {
                const __bf16 *Ph = reinterpret_cast<const __bf16 *>(phiB);
                for (int64_t a0 = 0; a0 < a.npad; a0 += 32) {
                    // B operand: X_p rows a0 + 8g + s at mode jw + c, split in three.
                    Split3 xr, xi;
#pragma unroll
                    for (int s = 0; s < 8; ++s) {
                        const int64_t ar = a0 + 8 * g + s;
                        float2 x = make_float2(0.f, 0.f);
                        if (ar < a.n) x = Xp[ar * a.Jpad + jw + c];
                        __bf16 h, mm, l;
                        split3(x.x, h, mm, l);
                        xr.h[s] = h; xr.m[s] = mm; xr.l[s] = l;
                        split3(x.y, h, mm, l);
                        xi.h[s] = h; xi.m[s] = mm; xi.l[s] = l;
                    }
#pragma unroll
                    for (int u = 0; u < NT1; ++u) {
                        const int64_t pidx = ((a0 / 8 + g) * a.npad + t0 + 16 * u + c) * 8;
                        Split3 pr, pi;
                        pr.h = *reinterpret_cast<const v8bf *>(Ph + 0 * N2 + pidx);
                        pr.m = *reinterpret_cast<const v8bf *>(Ph + 1 * N2 + pidx);
                        pr.l = *reinterpret_cast<const v8bf *>(Ph + 2 * N2 + pidx);
                        pi.h = *reinterpret_cast<const v8bf *>(Ph + 3 * N2 + pidx);
                        pi.m = *reinterpret_cast<const v8bf *>(Ph + 4 * N2 + pidx);
                        pi.l = *reinterpret_cast<const v8bf *>(Ph + 5 * N2 + pidx);
                        const Split3 pn = neg3(pi);
                        sr[u] = mm6(pr, xr, sr[u]);
                        sr[u] = mm6(pn, xi, sr[u]);
                        si[u] = mm6(pr, xi, si[u]);
                        si[u] = mm6(pi, xr, si[u]);
                    }
                }
            }

            // ---------------- divisor, division, weights (per element, FP64 divisor).
            real hr[NT1][4], hi[NT1][4];
#pragma unroll
            for (int u = 0; u < NT1; ++u)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t t = t0 + 16 * u + out_row<E>(r, g);
                    real vr = 0, vi = 0;
                    if (j_ok && t >= m && t < a.n) {
                        const double2 acc = add_fp64(lam_p, a.lam[t]);
                        const double2 d = divisor_fp64(acc, lam_j, a.eps);
                        const double w = (t == m) ? w_eq : w_gt;
                        scaled_quotient<E>(sr[u][r], si[u][r], d, w, a.tau2, vr, vi);
                    }
                    hr[u][r] = vr;
                    hi[u][r] = vi;
                }

            // ---------------- GEMM2: R[j][k] += sum_t h'[j][t] zeta[t][k].
            if constexpr (E == Eng::F64) {
                const double2 *Z = reinterpret_cast<const double2 *>(zetaB);
#pragma unroll
                for (int kt = 0; kt < NKTW; ++kt) {
                    if (kt0 + kt >= nkt) continue;
                    const int64_t k = int64_t(kt0 + kt) * 16 + c;
                    v4d accr, acci;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        accr[q] = pacc_r[kt][q];
                        acci[q] = pacc_i[kt][q];
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t t = t0 + out_row<E>(r, g);
                        // B = zeta[t][k] * zp[k]: the item is accumulated directly in FP64.
                        const double2 z = Z[t * a.npad + k];
                        const double br = z.x * zr[kt] - z.y * zi[kt];
                        const double bi = z.x * zi[kt] + z.y * zr[kt];
                        accr = mfma(hr[0][r], br, accr);
                        accr = mfma(-hi[0][r], bi, accr);
                        acci = mfma(hr[0][r], bi, acci);
                        acci = mfma(hi[0][r], br, acci);
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        pacc_r[kt][q] = accr[q];
                        pacc_i[kt][q] = acci[q];
                    }
                }
            } else if constexpr (E == Eng::F32) {
                const float2 *Z = reinterpret_cast<const float2 *>(zetaB);
#pragma unroll
                for (int kt = 0; kt < NKTW; ++kt) {
                    if (kt0 + kt >= nkt) continue;
                    const int64_t k = int64_t(kt0 + kt) * 16 + c;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t t = t0 + out_row<E>(r, g);
                        const float2 z = Z[t * a.npad + k];
                        rr[kt] = mfma(hr[0][r], z.x, rr[kt]);
                        rr[kt] = mfma(-hi[0][r], z.y, rr[kt]);
                        ri[kt] = mfma(hr[0][r], z.y, ri[kt]);
                        ri[kt] = mfma(hi[0][r], z.x, ri[kt]);
                    }
                }
            } else {
                // A operand: slot s < 4 <-> t0 + 4g + s (tile 0), s >= 4 <-> t0 + 16 + 4g + s - 4.
                Split3 ar_, ai_;
#pragma unroll
                for (int s = 0; s < 8; ++s) {
                    const int u = s >> 2, r = s & 3;
                    __bf16 h, mm, l;
                    split3(hr[u][r], h, mm, l);
                    ar_.h[s] = h; ar_.m[s] = mm; ar_.l[s] = l;
                    split3(hi[u][r], h, mm, l);
                    ai_.h[s] = h; ai_.m[s] = mm; ai_.l[s] = l;
                }
                const Split3 an_ = neg3(ai_);
                const __bf16 *Z = reinterpret_cast<const __bf16 *>(zetaB);
#pragma unroll
                for (int kt = 0; kt < NKTW; ++kt) {
                    if (kt0 + kt >= nkt) continue;
                    const int64_t k = int64_t(kt0 + kt) * 16 + c;
                    const int64_t z0 = zeta_frag_index(t0 + 4 * g, k, a.npad);
                    auto ld = [&](int pl) { return *reinterpret_cast<const v8bf *>(Z + pl * N2 + z0); };
                    Split3 zr_, zi_;
                    zr_.h = ld(0); zr_.m = ld(1); zr_.l = ld(2);
                    zi_.h = ld(3); zi_.m = ld(4); zi_.l = ld(5);
                    rr[kt] = mm6(ar_, zr_, rr[kt]);
                    rr[kt] = mm6(an_, zi_, rr[kt]);
                    ri[kt] = mm6(ar_, zi_, ri[kt]);
                    ri[kt] = mm6(ai_, zr_, ri[kt]);
                }
            }
        }
        // ---------------- item done: P += zp * R in FP64 (FP32 engines).
        if constexpr (E != Eng::F64) {
#pragma unroll
            for (int kt = 0; kt < NKTW; ++kt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const double vr = rr[kt][r], vi = ri[kt][r];
                    pacc_r[kt][r] += vr * zr[kt] - vi * zi[kt];
                    pacc_i[kt][r] += vr * zi[kt] + vi * zr[kt];
                }
        }
    }
    if (!wave_on) return;
    // ---------------- write this workgroup's partial.
    double2 *dst = a.parts + int64_t(blockIdx.x) * a.Jpad * a.n;
#pragma unroll
    for (int kt = 0; kt < NKTW; ++kt) {
        const int64_t k = int64_t(kt0 + kt) * 16 + c;
        if (kt0 + kt >= nkt || k >= a.n) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t j = jw + out_row<E>(r, g);
            if (j < a.Jpad) dst[j * a.n + k] = make_double2(pacc_r[kt][r], pacc_i[kt][r]);
        }
    }
}

// Partial sums in a fixed order, two levels: level 1 sums runs of 16 partials per element
// (coalesced over k), level 2 sums the level-1 results into rows [j0, j0+J) of P_M and
// adds P_M into the running sum over orders.

// One launch: 16 outputs (j, k) per workgroup, sixteen fixed ranges of slots per output
// summed by sixteen threads, the partial sums added in order -- the same result for any grid.
// For the last order (npf non-null) the finished sum over orders also gives the NPF entry
// NPF[k, j] = Phi[k, j] (delta Psi[j, k] + psum[j, k]) of Alg. 2 step 20 (the arithmetic of
// finalize_simt).
// Rows: partial row jj (computed mode j0 + jj) is output mode mm.row[jj]; a mode filled by
// conjugation (mm.conj[jj]) gets the conjugate P, sum and NPF entries.  scale multiplies P
// (1, or M! for Taylor-coefficient input).
__global__ void __launch_bounds__(256)
reduce_parts(const double2 *__restrict__ parts, int64_t nparts, int64_t Jpad, int64_t J,
             int64_t n, ModeMap mm, double scale, double2 *__restrict__ P,
             double2 *__restrict__ psum, int first, const double2 *__restrict__ Phi,
             const double2 *__restrict__ Psi, double delta, double2 *__restrict__ npf,
             double2 *__restrict__ inpf)
{
    __shared__ double2 part[16][16];
    const int64_t per = J * n;
    const int el = threadIdx.x & 15, grp = threadIdx.x >> 4;
    const int64_t chunk = (nparts + 15) / 16;
    for (int64_t e0 = int64_t(blockIdx.x) * 16; e0 < per; e0 += int64_t(gridDim.x) * 16) {
        const int64_t e = e0 + el;
        double sr = 0.0, si = 0.0;
        if (e < per) {
            const int64_t j = e / n, k = e % n;
            const int64_t b1 = (grp + 1) * chunk < nparts ? (grp + 1) * chunk : nparts;
            // Eight loads in flight, then their sums in slot order.
            for (int64_t b = grp * chunk; b < b1; b += 8) {
                double2 v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    v[u] = (b + u < b1) ? parts[((b + u) * Jpad + j) * n + k] : make_double2(0.0, 0.0);
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    sr += v[u].x;
                    si += v[u].y;
                }
            }
        }
        part[grp][el] = make_double2(sr, si);
        __syncthreads();
        if (grp == 0 && e < per) {
            double tr = 0.0, ti = 0.0;
            for (int q = 0; q < 16; ++q) {
                tr += part[q][el].x;
                ti += part[q][el].y;
            }
            tr *= scale;
            ti *= scale;
            const int64_t jj = e / n, k = e - jj * n;
            const int64_t j = mm.row[jj];
            if (inpf) {
                // Interaction factor of eq. (8): the sum is -sum_t h[j,t] prod zeta*_k[t_l].
                inpf[k * n + j] = cmul(Phi[k * n + j], make_double2(-tr, -ti));
                if (mm.conj[jj] != kNoRow) {
                    const int64_t jc = mm.conj[jj];
                    inpf[k * n + jc] = cmul(Phi[k * n + jc], make_double2(-tr, ti));
                }
            } else {
                P[j * n + k] = make_double2(tr, ti);
                double2 tot = make_double2(tr, ti);
                if (!first) {
                    const double2 o = psum[j * n + k];
                    tot = make_double2(o.x + tr, o.y + ti);
                }
                psum[j * n + k] = tot;
                if (npf) {
                    const double2 w = Psi[j * n + k];
                    double2 z = make_double2(delta * w.x, delta * w.y);
                    z = add_fp64(z, tot);
                    npf[k * n + j] = cmul(Phi[k * n + j], z);
                }
                if (mm.conj[jj] != kNoRow) {
                    const int64_t jc = mm.conj[jj];
                    const double2 totc = make_double2(tot.x, -tot.y);
                    P[jc * n + k] = make_double2(tr, -ti);
                    psum[jc * n + k] = totc;
                    if (npf) {
                        const double2 w = Psi[jc * n + k];
                        double2 z = make_double2(delta * w.x, delta * w.y);
                        z = add_fp64(z, totc);
                        npf[k * n + jc] = cmul(Phi[k * n + jc], z);
                    }
                }
            }
        }
        __syncthreads();
    }
}

template <Eng E, int NKTW, bool RES>
void launch_one(const dim3 &grid, size_t shm, const FusedArgs &fa, hipStream_t s)
{
    if (RES) {
        static bool attr = false;
        if (!attr) {
            (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&fused_last<E, NKTW, RES>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, int(kResidentBytes));
            attr = true;
        }
    }
    hipLaunchKernelGGL((fused_last<E, NKTW, RES>), grid, dim3(kThreads), shm, s, fa);
}

template <Eng E>
hipError_t launch_fused_eng(const FusedArgs &fa, int nkt, int64_t groups, hipStream_t s)
{
    int nktw = nkt <= 8 ? nkt : 8;
    if (nktw % 2) nktw += 1;
    const int kgroups = (nkt + nktw - 1) / nktw;
    const dim3 grid{unsigned(groups), unsigned((fa.Jpad + 63) / 64), unsigned(kgroups)};
    const int64_t rb = resident_bytes<E>(fa.npad);
    if (rb <= kResidentBytes && nktw <= 4) {
        if (nktw == 2) launch_one<E, 2, true>(grid, size_t(rb), fa, s);
        else launch_one<E, 4, true>(grid, size_t(rb), fa, s);
        return hipGetLastError();
    }
    switch (nktw) {
    case 2: launch_one<E, 2, false>(grid, 0, fa, s); break;
    case 4: launch_one<E, 4, false>(grid, 0, fa, s); break;
    case 6: launch_one<E, 6, false>(grid, 0, fa, s); break;
    default: launch_one<E, 8, false>(grid, 0, fa, s); break;
    }
    return hipGetLastError();
}

}  // namespace

// Workgroups along the items of the fused kernel (grid.x) for `items` items (all items
// when items < 0) and a block of Jpad modes.
static int64_t fused_gx(const npf_plan_s *p, int64_t items, int64_t Jpad)
{
    const bool tr = bf3_tr_fused_supported(p);
    const int64_t ipw = tr ? bf3_items_per_group(Jpad) : 1;
    const int64_t jgroups = (Jpad / 16 * ipw + 3) / 4;
    int64_t g = (bf3_small_supported(p) ? 256 : (tr ? 128 : 512)) / jgroups;
    if (g < 1) g = 1;
    if (items >= 0) {
        const int64_t need = (items + ipw - 1) / ipw;
        if (need < g) g = need > 0 ? need : 1;
    }
    return g;
}

// Partial-P slots written by the fused kernel for order M.
int64_t fused_groups(const npf_plan_s *p, int M)
{
    return fused_gx(p, p->U[M - 1], p->Jpad) *
           (bf3_tr_fused_supported(p) ? fused_bf3_tr_slices(p, p->Jpad) : 1);
}

// Most partial-P slots any order can write for a block of Jpad modes (workspace sizing).
int64_t fused_max_slots(const npf_plan_s *p, int64_t Jpad)
{
    return fused_gx(p, -1, Jpad) * (bf3_tr_fused_supported(p) ? fused_bf3_tr_slices(p, Jpad) : 1);
}

hipError_t launch_prepare(const npf_plan_s *p, const double *U, const double *V,
                          const double *lam, char *ws, hipStream_t s, const double *zadd)
{
    const int64_t N2 = p->npad * p->npad;
    char *base = ws + p->lay.phi;
    const bool sel = p->select;
    const int64_t work = N2 + p->tt.total + (sel ? p->nc * (p->n + 1) : 0);
    int64_t blocks = (work + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(prepare, dim3(unsigned(blocks)), dim3(256), 0, s,
                       reinterpret_cast<const double2 *>(V), reinterpret_cast<const double2 *>(U),
                       p->prob.delta, p->n, p->npad, p->prec, reinterpret_cast<double2 *>(base),
                       base + 16 * N2, base + 34 * N2, reinterpret_cast<float2 *>(base + 50 * N2),
                       reinterpret_cast<uint64_t *>(ws + p->lay.ttab), p->tt,
                       reinterpret_cast<const double2 *>(lam),
                       sel ? reinterpret_cast<double2 *>(ws + p->lay.msel) : nullptr, p->nc,
                       sel ? mode_map(p, 0, p->nc) : ModeMap{},
                       reinterpret_cast<const double2 *>(zadd));
    return hipGetLastError();
}

hipError_t launch_fused_last(const npf_plan_s *p, int M, int64_t j0, int64_t J, const double *lam,
                             char *ws, hipStream_t s)
{
    const int64_t N2 = p->npad * p->npad;
    char *base = ws + p->lay.phi;
    FusedArgs fa;
    fa.X = ws + p->lay.buf[(M - 1) % 2];
    fa.phiE = base + 16 * N2;
    fa.zetaE = base + 34 * N2;
    fa.zeta64 = reinterpret_cast<const double2 *>(base);
    fa.lam = reinterpret_cast<const double2 *>(lam);
    fa.lamj = reinterpret_cast<const double2 *>(lam_rows(p, lam, ws));
    fa.ptab = reinterpret_cast<const uint64_t *>(ws + p->lay.ttab) + p->tt.off[M - 1];
    fa.parts = reinterpret_cast<double2 *>(ws + p->lay.parts);
    fa.n = p->n;
    fa.npad = p->npad;
    fa.Jpad = p->Jpad;
    fa.J = J;
    fa.j0 = j0;
    fa.items = p->U[M - 1];
    fa.M = M;
    fa.eps = p->prob.eps;
    fa.tau2 = p->prob.tau * p->prob.tau;
    const int nkt = int(p->npad / 16);
    const int64_t groups = fused_gx(p, p->U[M - 1], p->Jpad);
    if (bf3_small_supported(p)) return launch_fused_bf3(p, M, j0, J, lam, ws, groups, s);
    if (bf3_tr_fused_supported(p)) return launch_fused_bf3_tr(p, M, j0, J, lam, ws, groups, s);
    switch (p->prec) {
    case NPF_FP64: return launch_fused_eng<Eng::F64>(fa, nkt, groups, s);
    case NPF_FP32: return launch_fused_eng<Eng::F32>(fa, nkt, groups, s);
    default: return launch_fused_eng<Eng::BF3>(fa, nkt, groups, s);
    }
}

// Workgroups along the items of the fused kernel of order M for the plan's block.
int64_t fused_default_groups(const npf_plan_s *p, int M) { return fused_gx(p, p->U[M - 1], p->Jpad); }

hipError_t launch_reduce_parts(const npf_plan_s *p, int M, int64_t j0, int64_t J, double *P,
                               double *psum, bool first, char *ws, hipStream_t s,
                               const NpfOut *fin, double *inpf)
{
    return launch_reduce_parts_n(p, fused_groups(p, M), j0, J, P, psum, first, ws, s, fin,
                                 p->a_scale[M], inpf);
}

hipError_t launch_reduce_parts_n(const npf_plan_s *p, int64_t nparts, int64_t j0, int64_t J,
                                 double *P, double *psum, bool first, char *ws, hipStream_t s,
                                 const NpfOut *fin, double scale, double *inpf)
{
    // The interaction factors need Phi; the other mode writes P and the running sum.
    if (inpf ? (!fin || !fin->V) : (!P || !psum)) return hipErrorInvalidValue;
    const int64_t per = J * p->n;
    int64_t wg = (per + 15) / 16;
    if (wg > 8192) wg = 8192;
    hipLaunchKernelGGL(reduce_parts, dim3(unsigned(wg)), dim3(256), 0, s,
                       reinterpret_cast<const double2 *>(ws + p->lay.parts), nparts, p->Jpad, J,
                       p->n, mode_map(p, j0, J), scale, reinterpret_cast<double2 *>(P),
                       reinterpret_cast<double2 *>(psum), first ? 1 : 0,
                       fin ? reinterpret_cast<const double2 *>(fin->V) : nullptr,
                       fin ? reinterpret_cast<const double2 *>(fin->U) : nullptr, p->prob.delta,
                       fin ? reinterpret_cast<double2 *>(fin->npf) : nullptr,
                       reinterpret_cast<double2 *>(inpf));
    return hipGetLastError();
}

}  // namespace npf
