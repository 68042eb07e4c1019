// Lower indices first for sparse derivative tensors (Alg. 2 steps 2-3, then step 4).
//
// When every row k of A_M involves at most smax states S(k), the lower-index mode products
// of row k only ever see Phi rows of S(k):
//   W[p][k][q] = sum_{b in S(k)^{M-1}} A_M[k, sort(b, S(k)[q])] prod_i Phi[b_i, p_i]
// for every sorted (M-1)-tuple p of modes, and the upper index then gives the input of the
// last mode product directly:
//   T_{M-1}[p][a][j] = sum_{k : a in S(k)} Psi[j, k] W[p][k][q(k, a)].
// This replaces the upper-index contraction and the M-2 chain stages, whose cost does not
// shrink with the sparsity.  Everything here is FP64; T_{M-1} is rounded once to the
// plan's storage precision.  Orders 2 and 3.
#include <algorithm>

#include "npf_device.h"
#include "npf_internal.h"

namespace npf {

namespace {

constexpr int kMaskWords = 4;      // n <= 256 states per bitmask row

// colex rank of a sorted tuple of local indices (< 8), length m <= 3.
__device__ __forceinline__ int local_rank(const int *x, int m)
{
    int r = 0;
    for (int i = 0; i < m; ++i) r += int(colex_term_c(x[i], i + 1));
    return r;
}

__device__ __forceinline__ int sorted3_rank(int u0, int u1, int u2)
{
    int tmp;
    if (u0 > u1) { tmp = u0; u0 = u1; u1 = tmp; }
    if (u1 > u2) { tmp = u1; u1 = u2; u2 = tmp; }
    if (u0 > u1) { tmp = u0; u0 = u1; u1 = tmp; }
    int loc[3] = {u0, u1, u2};
    return local_rank(loc, 3);
}

// Index of state a within S(k): the set bits of row k's mask below a.
__device__ __forceinline__ int mask_pos(const unsigned long long *m, int a)
{
    int q = 0;
    for (int w = 0; w < (a >> 6); ++w) q += __popcll(m[w]);
    const unsigned long long below = (a & 63) ? ((1ull << (a & 63)) - 1ull) : 0ull;
    return q + __popcll(m[a >> 6] & below);
}

// One workgroup per state k (grid.x): the states of row k's nonzeros (S(k), ascending,
// cnt[k] of them, -1 padded; over[k] = 1 when there are more than smax), and the dense
// table D_k[local colex rank] of the row's values over S(k).  Every workgroup scans the
// compressed columns for its own row, so no cross-workgroup step is needed.
__global__ void __launch_bounds__(1024)
tucker_rowk(const double *__restrict__ values, const int64_t *__restrict__ col_rank,
            const int64_t *__restrict__ col_ptr, const int32_t *__restrict__ row_k, int64_t ncols,
            int M, int64_t n, int smax, int32_t *__restrict__ S, int32_t *__restrict__ cnt,
            int32_t *__restrict__ over, double *__restrict__ D, int64_t UMs)
{
    __shared__ unsigned long long m[kMaskWords];
    __shared__ int64_t hits[512];          // (entry e) of this row, up to the list's capacity
    __shared__ int nhits;
    const int64_t k = blockIdx.x;
    if (threadIdx.x < kMaskWords) m[threadIdx.x] = 0ull;
    if (threadIdx.x == 0) nhits = 0;
    for (int64_t x = threadIdx.x; x < UMs; x += blockDim.x) D[k * UMs + x] = 0.0;
    __syncthreads();
    for (int64_t c = threadIdx.x; c < ncols; c += blockDim.x) {
        const int64_t e0 = col_ptr[c], e1 = col_ptr[c + 1];
        for (int64_t e = e0; e < e1; ++e)
            if (row_k[e] == k) {
                int32_t t[NPF_MAX_ORDER];
                colex_unrank(col_rank[c], M, n, t);
                for (int i = 0; i < M; ++i) atomicOr(&m[t[i] >> 6], 1ull << (t[i] & 63));
                const int h = atomicAdd(&nhits, 1);
                if (h < 512) hits[h] = (c << 20) | (e - e0);   // column, entry within it
            }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int q = 0;
        for (int a = 0; a < n; ++a)
            if ((m[a >> 6] >> (a & 63)) & 1ull) {
                if (q < smax) S[k * smax + q] = a;
                ++q;
            }
        // more states than declared, or more nonzeros than a row over smax states can hold
        over[k] = (q > smax || nhits > 512) ? 1 : 0;
        cnt[k] = q < smax ? q : smax;
        for (int r = q; r < smax; ++r) S[k * smax + r] = -1;
    }
    const int nh = nhits < 512 ? nhits : 512;
    for (int h = threadIdx.x; h < nh; h += blockDim.x) {
        const int64_t c = hits[h] >> 20, e = col_ptr[c] + (hits[h] & 0xfffff);
        int32_t t[NPF_MAX_ORDER];
        colex_unrank(col_rank[c], M, n, t);
        int loc[NPF_MAX_ORDER];
        bool ok = true;
        for (int i = 0; i < M; ++i) {
            loc[i] = mask_pos(m, t[i]);
            ok = ok && loc[i] < smax;
        }
        if (ok) D[k * UMs + local_rank(loc, M)] = values[e];
    }
}

// One workgroup per state a (grid.x): the inverse list inv[a][0 .. invcnt[a]) of packed
// (k << 8 | q) with S(k)[q] == a, in increasing k then q (a fixed order: the sums over them
// are deterministic).  The S table is scanned 256 entries at a time; matches are placed by
// a ballot prefix within each wave and the wave totals.
__global__ void __launch_bounds__(256)
tucker_inverse(const int32_t *__restrict__ S, int64_t n, int smax, int32_t *__restrict__ inv,
               int32_t *__restrict__ invcnt)
{
    __shared__ int wave_tot[4];
    const int64_t a = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t total = n * smax;
    int base = 0;
    for (int64_t x0 = 0; x0 < total; x0 += 256) {
        const int64_t x = x0 + threadIdx.x;
        const bool hit = x < total && S[x] == a;
        const unsigned long long bal = __ballot(hit);
        const int before = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wave_tot[wave] = __popcll(bal);
        __syncthreads();
        int off = base;
        for (int w = 0; w < wave; ++w) off += wave_tot[w];
        if (hit) inv[a * n + off + before] = int32_t(((x / smax) << 8) | (x % smax));
        base += wave_tot[0] + wave_tot[1] + wave_tot[2] + wave_tot[3];
        __syncthreads();
    }
    if (threadIdx.x == 0) invcnt[a] = base;
}

// Order 2: W[t][k][q] = sum_{b < s} D_k[sort(b, q)] Phi[S(k)[b], t].
// Order 3, first half: Y[k][b0][t][q] = sum_{b1 < s} D_k[sort(b0, b1, q)] Phi[S(k)[b1], t].
// grid.y = k; row k's Phi rows and D_k in LDS; one thread per (t, q).
template <int M>
__global__ void __launch_bounds__(256)
tucker_rows_first(const double2 *__restrict__ Phi, int64_t n, const int32_t *__restrict__ S,
                  const int32_t *__restrict__ cnt, int smax, const double *__restrict__ D,
                  int64_t UMs, double2 *__restrict__ out)
{
    __shared__ double2 phiL[kTuckerMaxSupport * 256];   // [b][t]
    __shared__ double DL[128];                          // binom(8 + 3 - 1, 3) = 120 at most
    const int64_t k = blockIdx.y;
    const int s = cnt[k];
    for (int64_t x = threadIdx.x; x < s * n; x += blockDim.x) {
        const int64_t b = x / n, t = x % n;
        phiL[b * n + t] = Phi[int64_t(S[k * smax + b]) * n + t];
    }
    for (int64_t x = threadIdx.x; x < UMs; x += blockDim.x) DL[x] = D[k * UMs + x];
    __syncthreads();
    const int q = threadIdx.x % kTuckerMaxSupport;
    constexpr int TPB = 256 / kTuckerMaxSupport;
    for (int64_t t = int64_t(blockIdx.x) * TPB + threadIdx.x / kTuckerMaxSupport; t < n;
         t += int64_t(gridDim.x) * TPB) {
        if (q >= smax) continue;
        if constexpr (M == 2) {
            double2 acc = make_double2(0.0, 0.0);
            for (int b = 0; b < s && q < s; ++b) {
                int loc[2] = {b < q ? b : q, b < q ? q : b};
                const double v = DL[local_rank(loc, 2)];
                const double2 f = phiL[b * n + t];
                acc.x += v * f.x;
                acc.y += v * f.y;
            }
            out[(t * n + k) * smax + q] = acc;
        } else {
            for (int b0 = 0; b0 < smax; ++b0) {
                double2 acc = make_double2(0.0, 0.0);
                for (int b1 = 0; b1 < s && b0 < s && q < s; ++b1) {
                    const double v = DL[sorted3_rank(b0, b1, q)];
                    const double2 f = phiL[b1 * n + t];
                    acc.x += v * f.x;
                    acc.y += v * f.y;
                }
                out[((k * smax + b0) * n + t) * smax + q] = acc;
            }
        }
    }
}

// Order 3, second half: W[rank(p0, p1)][k][q] = sum_{b0 < s} Phi[S(k)[b0], p0] Y[k][b0][p1][q].
__global__ void __launch_bounds__(256)
tucker_w3(const uint64_t *__restrict__ ptab, int64_t np, const double2 *__restrict__ Phi, int64_t n,
          const int32_t *__restrict__ S, const int32_t *__restrict__ cnt, int smax,
          const double2 *__restrict__ Y, double2 *__restrict__ W)
{
    __shared__ double2 phiL[kTuckerMaxSupport * 256];
    const int64_t k = blockIdx.y;
    const int s = cnt[k];
    for (int64_t x = threadIdx.x; x < s * n; x += blockDim.x) {
        const int64_t b = x / n, t = x % n;
        phiL[b * n + t] = Phi[int64_t(S[k * smax + b]) * n + t];
    }
    __syncthreads();
    const int q = threadIdx.x % kTuckerMaxSupport;
    constexpr int TPB = 256 / kTuckerMaxSupport;
    const double2 *Yk = Y + k * smax * n * smax;
    for (int64_t rp = int64_t(blockIdx.x) * TPB + threadIdx.x / kTuckerMaxSupport; rp < np;
         rp += int64_t(gridDim.x) * TPB) {
        if (q >= smax) continue;
        const uint64_t pk = ptab[rp];
        const int p0 = tuple_at(pk, 0), p1 = tuple_at(pk, 1);
        double2 y[kTuckerMaxSupport];
#pragma unroll
        for (int b0 = 0; b0 < kTuckerMaxSupport; ++b0)     // independent loads, issued together
            y[b0] = (b0 < s && q < s) ? Yk[(b0 * n + p1) * smax + q] : make_double2(0.0, 0.0);
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll
        for (int b0 = 0; b0 < kTuckerMaxSupport; ++b0)
            if (b0 < s) acc = add_fp64(acc, cmul(phiL[b0 * n + p0], y[b0]));
        W[(rp * n + k) * smax + q] = acc;
    }
}

// T[rp][a][jj] = sum_{(k,q) in inv(a)} Psi[j0 + jj, k] W[rp][k][q] for jj < J (0 for the
// padding).  grid.y: 16-mode tiles with their Psi^T columns in LDS; per prefix rp the
// workgroup stages W[rp] and writes its n x JT outputs.  A row marked as having more
// states than declared makes every entry NaN.
template <typename OutC, int JT>
__global__ void __launch_bounds__(256)
tucker_psi(const double2 *__restrict__ W, int64_t np, int64_t n, int smax,
           const int32_t *__restrict__ inv, const int32_t *__restrict__ invcnt,
           const double2 *__restrict__ Psi, int64_t j0, int64_t J, int64_t Jpad,
           const int32_t *__restrict__ over, OutC *__restrict__ T)
{
    extern __shared__ __align__(16) char lds[];
    double2 *psiT = reinterpret_cast<double2 *>(lds);                    // [k][JT]
    double2 *Wb = psiT + n * JT;                                        // [k][smax]
    int32_t *iptr = reinterpret_cast<int32_t *>(Wb + n * smax);         // [n + 1]
    int32_t *ilist = iptr + n + 1;                                      // [n * smax]
    const int jt = int(blockIdx.y);
    for (int64_t x = threadIdx.x; x < n * JT; x += blockDim.x) {        // coalesced along k
        const int64_t jl = x / n, k = x % n, j = int64_t(jt) * JT + jl;
        psiT[k * JT + jl] = j < J ? Psi[(j0 + j) * n + k] : make_double2(0.0, 0.0);
    }
    // CSR of the inverse lists in LDS: exclusive scan of the counts (n <= 256 entries).
    __shared__ int32_t scan[256];
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    const int c0 = threadIdx.x < n ? invcnt[threadIdx.x] : 0;
    scan[threadIdx.x] = c0;
    __syncthreads();
    if (threadIdx.x < n && over[threadIdx.x]) atomicOr(&bad, 1);
    for (int d = 1; d < 256; d <<= 1) {
        const int v = threadIdx.x >= d ? scan[threadIdx.x - d] : 0;
        __syncthreads();
        scan[threadIdx.x] += v;
        __syncthreads();
    }
    if (threadIdx.x < n) iptr[threadIdx.x + 1] = scan[threadIdx.x];
    if (threadIdx.x == 0) iptr[0] = 0;
    __syncthreads();
    for (int x = threadIdx.x; x < iptr[n]; x += blockDim.x) {   // independent loads
        int lo = 0, hi = int(n) - 1;                                // a with iptr[a] <= x < iptr[a+1]
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (iptr[mid] <= x) lo = mid; else hi = mid - 1;
        }
        ilist[x] = inv[int64_t(lo) * n + (x - iptr[lo])];
    }
    const bool poison = bad != 0;
    constexpr int AR = 256 / JT;            // a-rows per pass
    const int jl = threadIdx.x % JT, arow = threadIdx.x / JT;
    const int64_t jj = int64_t(jt) * JT + jl;
    using real = decltype(OutC{}.x);
    for (int64_t rp = blockIdx.x; rp < np; rp += gridDim.x) {
        __syncthreads();                       // the previous prefix's W block is consumed
        const double2 *src = W + rp * n * smax;
        for (int64_t x = threadIdx.x; x < n * smax; x += blockDim.x) Wb[x] = src[x];
        __syncthreads();
        for (int64_t a = arow; a < n; a += AR) {
            double2 acc = make_double2(0.0, 0.0);
            const int i1 = iptr[a + 1];
            int i = iptr[a];
            for (; i + 4 <= i1; i += 4) {          // four terms with independent loads
                double2 w[4], ps[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int kq = ilist[i + u];
                    w[u] = Wb[(kq >> 8) * smax + (kq & 255)];
                    ps[u] = psiT[(kq >> 8) * JT + jl];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    acc.x += w[u].x * ps[u].x - w[u].y * ps[u].y;
                    acc.y += w[u].x * ps[u].y + w[u].y * ps[u].x;
                }
            }
            for (; i < i1; ++i) {
                const int kq = ilist[i];
                const int k = kq >> 8, q = kq & 255;
                const double2 w = Wb[k * smax + q];
                const double2 ps = psiT[k * JT + jl];
                acc.x += w.x * ps.x - w.y * ps.y;
                acc.y += w.x * ps.y + w.y * ps.x;
            }
            if (poison) acc = make_double2(__builtin_nan(""), __builtin_nan(""));
            if (jj < Jpad) T[(rp * n + a) * Jpad + jj] = OutC{real(acc.x), real(acc.y)};
        }
    }
}

}  // namespace

bool tucker_route(const npf_plan_s *p, int M)
{
    // Order 3 saves the upper-index contraction and two chain stages of n U_1 U_2 per mode;
    // order 2 only the single stage (n^3 per mode), which pays for the per-row tables only
    // for larger n.
    // The split-BF16 chain stages are fast enough below about 64 states that the per-row
    // tables do not pay for themselves there; the FP64 stages are not.
    const bool bound = p->prob.support_max >= 1 && p->prob.support_max <= kTuckerMaxSupport;
    const bool o3 = M == 3 && (p->n > 64 || p->prec == NPF_FP64);
    return bound && p->n <= 256 && (o3 || (M == 2 && p->n > 96));
}

bool tucker_supported(const npf_plan_s *p, const npf_tensor *A, int M)
{
    return A->kind == NPF_SRC_SPARSE && tucker_route(p, M);
}

hipError_t launch_tucker_rows(const npf_plan_s *p, int M, const npf_tensor *A, const double *V,
                              char *ws, hipStream_t s)
{
    const hipError_t e = launch_tucker_support(p, M, A, ws, s);
    return e != hipSuccess ? e : launch_tucker_w(p, M, V, ws, s);
}

hipError_t launch_tucker_support(const npf_plan_s *p, int M, const npf_tensor *A, char *ws,
                                 hipStream_t s)
{
    const int smax = p->prob.support_max;
    const TuckerLayout &t = p->lay.tk;
    int32_t *S = reinterpret_cast<int32_t *>(ws + t.S);
    int32_t *cnt = reinterpret_cast<int32_t *>(ws + t.cnt);
    int32_t *over = reinterpret_cast<int32_t *>(ws + t.over);
    int32_t *inv = reinterpret_cast<int32_t *>(ws + t.inv);
    int32_t *invcnt = reinterpret_cast<int32_t *>(ws + t.invcnt);
    double *D = reinterpret_cast<double *>(ws + t.D);
    const int64_t UMs = binom(smax + M - 1, M);
    hipLaunchKernelGGL(tucker_rowk, dim3(unsigned(p->n)), dim3(1024), 0, s, A->values, A->col_rank,
                       A->col_ptr, A->row_k, A->ncols, M, p->n, smax, S, cnt, over, D, UMs);
    hipLaunchKernelGGL(tucker_inverse, dim3(unsigned(p->n)), dim3(256), 0, s, S, p->n, smax, inv,
                       invcnt);
    return hipGetLastError();
}

hipError_t launch_tucker_w(const npf_plan_s *p, int M, const double *V, char *ws, hipStream_t s)
{
    const int smax = p->prob.support_max;
    const TuckerLayout &t = p->lay.tk;
    const int32_t *S = reinterpret_cast<const int32_t *>(ws + t.S);
    const int32_t *cnt = reinterpret_cast<const int32_t *>(ws + t.cnt);
    const double *D = reinterpret_cast<const double *>(ws + t.D);
    const int64_t UMs = binom(smax + M - 1, M);
    const double2 *Phi = reinterpret_cast<const double2 *>(V);
    double2 *W = reinterpret_cast<double2 *>(ws + t.W);
    constexpr int TPB = 256 / kTuckerMaxSupport;
    const dim3 grid_t{unsigned((p->n + TPB - 1) / TPB), unsigned(p->n), 1u};
    if (M == 2) {
        hipLaunchKernelGGL(tucker_rows_first<2>, grid_t, dim3(256), 0, s, Phi, p->n, S, cnt, smax, D,
                           UMs, W);
        return hipGetLastError();
    }
    double2 *Y = reinterpret_cast<double2 *>(ws + t.Y);
    hipLaunchKernelGGL(tucker_rows_first<3>, grid_t, dim3(256), 0, s, Phi, p->n, S, cnt, smax, D,
                       UMs, Y);
    const int64_t np = p->U[M - 1];
    const uint64_t *ptab = reinterpret_cast<const uint64_t *>(ws + p->lay.ttab) + p->tt.off[M - 1];
    int64_t gx = (np + TPB - 1) / TPB;
    const int64_t cap = std::max<int64_t>(1, 8192 / p->n);
    if (gx > cap) gx = cap;
    hipLaunchKernelGGL(tucker_w3, dim3(unsigned(gx), unsigned(p->n), 1u), dim3(256), 0, s, ptab, np,
                       Phi, p->n, S, cnt, smax, Y, W);
    return hipGetLastError();
}

hipError_t launch_tucker_psi(const npf_plan_s *p, int M, int64_t j0, int64_t J, const double *U,
                             char *ws, hipStream_t s)
{
    const TuckerLayout &t = p->lay.tk;
    const int smax = p->prob.support_max;
    const int64_t np = p->U[M - 1];
    // 64 modes per workgroup while Psi^T of the tile fits comfortably in LDS, else 16.
    const int jtile = (p->n <= 128) ? 32 : 16;
    const int64_t gy = (p->Jpad + jtile - 1) / jtile;
    int64_t gx = np;
    const int64_t cap = std::max<int64_t>(1, 1024 / gy);
    if (gx > cap) gx = cap;
    const dim3 grid{unsigned(gx), unsigned(gy), 1u};
    const size_t shm = size_t(p->n) * jtile * sizeof(double2) + size_t(p->n * smax) * sizeof(double2) +
                       size_t(p->n + 1 + p->n * smax) * sizeof(int32_t);
    void *dst = ws + p->lay.buf[(M - 1) % 2];
    const double2 *W = reinterpret_cast<const double2 *>(ws + t.W);
    const int32_t *inv = reinterpret_cast<const int32_t *>(ws + t.inv);
    const int32_t *invcnt = reinterpret_cast<const int32_t *>(ws + t.invcnt);
    const int32_t *over = reinterpret_cast<const int32_t *>(ws + t.over);
    const double2 *Psi = reinterpret_cast<const double2 *>(U);
#define NPF_TUCKER_PSI(C_, JT_)                                                                \
    {                                                                                          \
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&tucker_psi<C_, JT_>),         \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(shm));        \
        hipLaunchKernelGGL((tucker_psi<C_, JT_>), grid, dim3(256), shm, s, W, np, p->n, smax,   \
                           inv, invcnt, Psi, j0, J, p->Jpad, over, static_cast<C_ *>(dst)); \
    }
    if (p->prec == NPF_FP64) {
        if (jtile == 32) NPF_TUCKER_PSI(double2, 32) else NPF_TUCKER_PSI(double2, 16)
    } else {
        if (jtile == 32) NPF_TUCKER_PSI(float2, 32) else NPF_TUCKER_PSI(float2, 16)
    }
#undef NPF_TUCKER_PSI
    return hipGetLastError();
}

}  // namespace npf
