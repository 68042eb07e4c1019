// Upper-index contraction on MFMA for dense derivative tensors (Alg. 2 step 4, done
// first):  T_0[r][jj] = sum_k A_M[k][r] Psi[j0 + jj][k]  for every sorted tuple r.
// (The split-BF16 path uses psi_a_bf3 below where Psi^T's six planes fit in LDS.)
// A_M is real and read once per output-mode block, so the kernel is bound by the HBM
// stream of A_M; Psi^T for the block (n x Jpad complex) stays in LDS for the whole launch
// and each workgroup sweeps 64-row tiles of r.  FP64 MFMA for the FP64 and split-BF16
// paths (the split path stores the result in FP32: one rounding of an FP64 sum over the n
// states), FP32 MFMA for the FP32 path.  For a hash-generated tensor the A_M entries are
// generated in registers where the stored ones would be loaded.
#include "npf_device.h"
#include "npf_internal.h"
#include "npf_mfma.h"

namespace npf {

namespace {

constexpr int kThreads = 256;   // 4 waves, 16 rows r each

// Where A_M comes from: stored values, or the hash generator.
struct ASrc {
    const double *A;
    uint64_t seed;
    double scale;
    int M;
};

template <Eng E, int NJT, bool HASH, typename OutC>
__global__ void __launch_bounds__(kThreads)
psi_a_mfma(ASrc src, const double2 *__restrict__ Psi, int64_t n, int64_t UM, int64_t j0,
           int64_t J, int64_t Jpad, void *__restrict__ out_)
{
    using T = EngT<E>;
    using acc_t = typename T::acc;
    using real = typename T::real;
    using cplx = typename T::cplx;
    extern __shared__ __align__(16) char lds[];
    cplx *L = reinterpret_cast<cplx *>(lds);         // Psi^T[k][jj], zero for jj >= J
    const int64_t npad32 = (n + 31) / 32 * 32;
    for (int64_t x = threadIdx.x; x < npad32 * Jpad; x += blockDim.x) {
        const int64_t k = x / Jpad, jj = x % Jpad;
        double2 v = make_double2(0.0, 0.0);
        if (k < n && jj < J) v = Psi[(j0 + jj) * n + k];
        L[x] = cplx{real(v.x), real(v.y)};
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, c = lane & 15;
    OutC *out = static_cast<OutC *>(out_);
    using out_real = decltype(OutC{}.x);
    for (int64_t r0 = int64_t(blockIdx.x) * 64 + wave * 16; r0 < UM; r0 += int64_t(gridDim.x) * 64) {
        const int64_t r = r0 + c;
        const bool r_ok = r < UM;
        acc_t ar[NJT], ai[NJT];
#pragma unroll
        for (int u = 0; u < NJT; ++u) ar[u] = ai[u] = acc_t{0, 0, 0, 0};
        for (int64_t k0 = 0; k0 < npad32; k0 += 32) {
            // A operand: A^T[r][k] = A[k][r] (lanes of a group read consecutive r); the
            // eight loads of a 32-wide chunk are issued together.
            real av[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int64_t k = k0 + 4 * q + g;
                if constexpr (HASH)
                    av[q] = (r_ok && k < n) ? real(hash_entry(src.seed, src.scale, src.M, k, r))
                                            : real(0);
                else
                    av[q] = (r_ok && k < n) ? real(src.A[k * UM + r]) : real(0);
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int64_t k = k0 + 4 * q + g;
#pragma unroll
                for (int u = 0; u < NJT; ++u) {
                    const cplx p = L[k * Jpad + u * 16 + c];      // B operand: Psi^T[k][jj]
                    ar[u] = mfma(av[q], p.x, ar[u]);
                    ai[u] = mfma(av[q], p.y, ai[u]);
                }
            }
        }
        // D[row = r0 + out_row][col = jj]: lanes of a group write consecutive jj.
#pragma unroll
        for (int u = 0; u < NJT; ++u)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t rr = r0 + out_row<E>(q, g);
                if (rr < UM)
                    out[rr * Jpad + u * 16 + c] = OutC{out_real(ar[u][q]), out_real(ai[u][q])};
            }
    }
}

// The same contraction for the split-BF16 path on the BF16 matrix cores: A_M rounded to FP32
// and split exactly in three BF16 terms in registers, Psi^T (rounded to FP32) as six BF16
// planes in LDS laid out [plane][k/8][jj][k%8] so that a B fragment is one 16-byte read, six
// of the nine term products per pair, the hi*hi sum kept apart from the five smaller ones.
// Eight waves of 16 rows r; the next K-chunk of A is loaded while the current one computes.
template <int NJT, bool HASH>
__global__ void __launch_bounds__(512)
psi_a_bf3(ASrc src, const double2 *__restrict__ Psi, int64_t n, int64_t UM, int64_t j0,
          int64_t J, int64_t Jpad, float2 *__restrict__ out)
{
    extern __shared__ __align__(16) char lds[];
    __bf16 *L = reinterpret_cast<__bf16 *>(lds);
    const int64_t npad32 = (n + 31) / 32 * 32;
    const int64_t PL = npad32 * Jpad;             // elements per plane
    for (int64_t x = threadIdx.x; x < PL; x += blockDim.x) {
        const int64_t k = x / Jpad, jj = x % Jpad;
        double2 v = make_double2(0.0, 0.0);
        if (k < n && jj < J) v = Psi[(j0 + jj) * n + k];
        const int64_t e = ((k / 8) * Jpad + jj) * 8 + (k % 8);
        __bf16 h, m, l;
        split3(float(v.x), h, m, l);
        L[0 * PL + e] = h; L[1 * PL + e] = m; L[2 * PL + e] = l;
        split3(float(v.y), h, m, l);
        L[3 * PL + e] = h; L[4 * PL + e] = m; L[5 * PL + e] = l;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int nn = int(n);
    for (int64_t r0 = int64_t(blockIdx.x) * 128 + wave * 16; r0 < UM; r0 += int64_t(gridDim.x) * 128) {
        const int64_t r = r0 + c;
        const bool r_ok = r < UM;
        // A^T[r][k] for k = k0 + 8g + s (lanes of a group read consecutive r).
        auto load = [&](int64_t k0, double (&av)[8]) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int k = int(k0) + 8 * g + q;
                if constexpr (HASH)
                    av[q] = (r_ok && k < nn) ? hash_entry(src.seed, src.scale, src.M, k, r) : 0.0;
                else
                    av[q] = (r_ok && k < nn) ? src.A[int64_t(k) * UM + r] : 0.0;
            }
        };
        v4f hr[NJT], lr[NJT], hi[NJT], li[NJT];
#pragma unroll
        for (int u = 0; u < NJT; ++u) hr[u] = lr[u] = hi[u] = li[u] = v4f{0, 0, 0, 0};
        double cur[8];
        load(0, cur);
        for (int64_t k0 = 0; k0 < npad32; k0 += 32) {
            double nxt[8];
            if (!HASH && k0 + 32 < npad32) load(k0 + 32, nxt);
            float af[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) af[q] = float(cur[q]);
            const Split3 as = split8(af);
#pragma unroll
            for (int u = 0; u < NJT; ++u) {
                const int64_t e = ((k0 / 8 + g) * Jpad + u * 16 + c) * 8;
                Split3 br, bi;
                br.h = *reinterpret_cast<const v8bf *>(L + 0 * PL + e);
                br.m = *reinterpret_cast<const v8bf *>(L + 1 * PL + e);
                br.l = *reinterpret_cast<const v8bf *>(L + 2 * PL + e);
                bi.h = *reinterpret_cast<const v8bf *>(L + 3 * PL + e);
                bi.m = *reinterpret_cast<const v8bf *>(L + 4 * PL + e);
                bi.l = *reinterpret_cast<const v8bf *>(L + 5 * PL + e);
                mm6s(as, br, hr[u], lr[u]);
                mm6s(as, bi, hi[u], li[u]);
            }
            if (k0 + 32 < npad32) {
                if constexpr (HASH) load(k0 + 32, cur);
                else {
#pragma unroll
                    for (int q = 0; q < 8; ++q) cur[q] = nxt[q];
                }
            }
        }
        // D[row = r0 + 4g + q][col = jj]: lanes of a group write consecutive jj.
#pragma unroll
        for (int u = 0; u < NJT; ++u)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t rr = r0 + 4 * g + q;
                if (rr < UM)
                    out[rr * Jpad + u * 16 + c] = make_float2(hr[u][q] + lr[u][q], hi[u][q] + li[u][q]);
            }
    }
}

template <int NJT>
hipError_t launch_bf3(const ASrc &src, bool hashed, const double2 *Psi, int64_t n, int64_t UM,
                      int64_t j0, int64_t J, int64_t Jpad, void *out, hipStream_t s)
{
    const int64_t npad32 = (n + 31) / 32 * 32;
    const size_t shm = size_t(npad32 * Jpad) * 12;
    int64_t tiles = (UM + 127) / 128;
    const int64_t cap = hashed ? 4096 : 1024;
    if (tiles > cap) tiles = cap;
    float2 *o = static_cast<float2 *>(out);
    if (hashed) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&psi_a_bf3<NJT, true>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(shm));
        hipLaunchKernelGGL((psi_a_bf3<NJT, true>), dim3(unsigned(tiles)), dim3(512), shm, s, src,
                           Psi, n, UM, j0, J, Jpad, o);
    } else {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&psi_a_bf3<NJT, false>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(shm));
        hipLaunchKernelGGL((psi_a_bf3<NJT, false>), dim3(unsigned(tiles)), dim3(512), shm, s, src,
                           Psi, n, UM, j0, J, Jpad, o);
    }
    return hipGetLastError();
}

template <Eng E, int NJT, bool HASH, typename OutC>
hipError_t launch_one(const ASrc &src, const double2 *Psi, int64_t n, int64_t UM, int64_t j0,
                      int64_t J, int64_t Jpad, void *out, hipStream_t s)
{
    const int64_t npad32 = (n + 31) / 32 * 32;
    const size_t shm = size_t(npad32 * Jpad) * sizeof(typename EngT<E>::cplx);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&psi_a_mfma<E, NJT, HASH, OutC>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(shm));
    // Generation costs ~40 integer ops per entry: more workgroups to hide it.
    int64_t tiles = (UM + 63) / 64;
    const int64_t cap = HASH ? 4096 : 1024;
    if (tiles > cap) tiles = cap;
    hipLaunchKernelGGL((psi_a_mfma<E, NJT, HASH, OutC>), dim3(unsigned(tiles)), dim3(kThreads),
                       shm, s, src, Psi, n, UM, j0, J, Jpad, out);
    return hipGetLastError();
}

template <Eng E, int NJT, typename OutC = typename EngT<E>::cplx>
hipError_t launch(const ASrc &src, bool hashed, const double2 *Psi, int64_t n, int64_t UM,
                  int64_t j0, int64_t J, int64_t Jpad, void *out, hipStream_t s)
{
    if (hashed) return launch_one<E, NJT, true, OutC>(src, Psi, n, UM, j0, J, Jpad, out, s);
    return launch_one<E, NJT, false, OutC>(src, Psi, n, UM, j0, J, Jpad, out, s);
}

}  // namespace

bool psi_a_mfma_supported(const npf_plan_s *p)
{
    // Psi^T of the block must fit in LDS and the block must be at most 128 modes.
    const int64_t npad32 = (p->n + 31) / 32 * 32;
    const int64_t bytes = npad32 * p->Jpad * (p->prec == NPF_FP32 ? 8 : 16);
    return p->Jpad <= 128 && bytes <= 144 * 1024;
}

hipError_t launch_psi_a_mfma(const ChainArgs &a)
{
    const npf_plan_s &p = *a.plan;
    const int64_t UM = p.U[a.M];
    void *dst = a.ws + p.lay.buf[0];
    const double2 *Psi = reinterpret_cast<const double2 *>(a.U);
    const int njt = int(p.Jpad / 16);
    const ASrc src{a.A->values, a.A->seed, a.A->scale, a.M};
    const bool hashed = a.A->kind == NPF_SRC_HASH;
#define NPF_PSI_CASE(E_, K_)                                                                 \
    if (njt == K_) return launch<E_, K_>(src, hashed, Psi, p.n, UM, a.j0, a.J, p.Jpad, dst, \
                                         a.stream);
    if (p.prec == NPF_FP64) {
        NPF_PSI_CASE(Eng::F64, 1) NPF_PSI_CASE(Eng::F64, 2) NPF_PSI_CASE(Eng::F64, 3)
        NPF_PSI_CASE(Eng::F64, 4) NPF_PSI_CASE(Eng::F64, 5) NPF_PSI_CASE(Eng::F64, 6)
        NPF_PSI_CASE(Eng::F64, 7) NPF_PSI_CASE(Eng::F64, 8)
    } else if (p.prec == NPF_BF16X3 && (p.n + 31) / 32 * 32 * p.Jpad * 12 <= 144 * 1024) {
#define NPF_PSI_CASE_BF3(K_) \
    if (njt == K_) return launch_bf3<K_>(src, hashed, Psi, p.n, UM, a.j0, a.J, p.Jpad, dst, a.stream);
        NPF_PSI_CASE_BF3(1) NPF_PSI_CASE_BF3(2) NPF_PSI_CASE_BF3(3) NPF_PSI_CASE_BF3(4)
        NPF_PSI_CASE_BF3(5) NPF_PSI_CASE_BF3(6) NPF_PSI_CASE_BF3(7) NPF_PSI_CASE_BF3(8)
#undef NPF_PSI_CASE_BF3
    } else if (p.prec == NPF_BF16X3) {
#define NPF_PSI_CASE64(K_)                                                                   \
    if (njt == K_) return launch<Eng::F64, K_, float2>(src, hashed, Psi, p.n, UM, a.j0, a.J, \
                                                       p.Jpad, dst, a.stream);
        NPF_PSI_CASE64(1) NPF_PSI_CASE64(2) NPF_PSI_CASE64(3) NPF_PSI_CASE64(4)
        NPF_PSI_CASE64(5) NPF_PSI_CASE64(6) NPF_PSI_CASE64(7) NPF_PSI_CASE64(8)
#undef NPF_PSI_CASE64
    } else {
        NPF_PSI_CASE(Eng::F32, 1) NPF_PSI_CASE(Eng::F32, 2) NPF_PSI_CASE(Eng::F32, 3)
        NPF_PSI_CASE(Eng::F32, 4) NPF_PSI_CASE(Eng::F32, 5) NPF_PSI_CASE(Eng::F32, 6)
        NPF_PSI_CASE(Eng::F32, 7) NPF_PSI_CASE(Eng::F32, 8)
    }
#undef NPF_PSI_CASE
    return hipErrorInvalidValue;
}

}  // namespace npf
