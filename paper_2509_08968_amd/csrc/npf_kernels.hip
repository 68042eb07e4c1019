// Straightforward (SIMT) kernels of the hot path: the upper-index contraction, one stage
// of the lower-index chain, the last stage into C, the divisor / division, the reduction
// to P and the NPF assembly.  These serve the step-by-step entry points and are the
// reference structure for the fused MFMA kernels.  The mixed paths store their results in
// FP32 but these kernels sum in FP64 (a sequential FP32 sum over 150 states lost 3e-7).
#include "npf_device.h"
#include "npf_internal.h"

namespace npf {

namespace {

constexpr int kThreads = 256;

template <typename T> struct Cplx;
template <> struct Cplx<double> { using type = double2; };
template <> struct Cplx<float> { using type = float2; };

__device__ __forceinline__ double2 to_d2(double2 v) { return v; }
__device__ __forceinline__ double2 to_d2(float2 v) { return make_double2(v.x, v.y); }
template <typename C> __device__ __forceinline__ C from_d2(double2 v);
template <> __device__ __forceinline__ double2 from_d2<double2>(double2 v) { return v; }
template <> __device__ __forceinline__ float2 from_d2<float2>(double2 v)
{
    return make_float2(float(v.x), float(v.y));
}

// ---------------------------------------------------------------- upper index first
// T_0[r][jj] = sum_k A_M[k][r] Psi[j0 + jj][k] for jj < J (zero for the padded modes).
template <typename C, typename Acc>
__global__ void __launch_bounds__(kThreads)
psi_a_dense(const double *__restrict__ A, const double2 *__restrict__ Psi, int64_t n, int64_t UM,
            int64_t j0, int64_t J, int64_t Jpad, C *__restrict__ out, int hashed, uint64_t seed,
            double scale, int M)
{
    const int64_t total = UM * Jpad;
    for (int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < total;
         x += int64_t(gridDim.x) * blockDim.x) {
        const int64_t r = x / Jpad, jj = x % Jpad;
        Acc re = 0, im = 0;
        if (jj < J) {
            const double2 *psi = Psi + (j0 + jj) * n;
            for (int64_t k = 0; k < n; ++k) {
                const Acc a = Acc(hashed ? hash_entry(seed, scale, M, k, r) : A[k * UM + r]);
                const double2 w = psi[k];
                re += a * Acc(w.x);
                im += a * Acc(w.y);
            }
        }
        out[x] = from_d2<C>(make_double2(double(re), double(im)));
    }
}


// Rows [k0, k0 + rows) of a hash-generated tensor, materialised: out[(k - k0)*UM + r].
__global__ void __launch_bounds__(kThreads)
hash_fill(double *__restrict__ out, uint64_t seed, double scale, int M, int64_t k0, int64_t rows,
          int64_t UM)
{
    const int64_t total = rows * UM;
    for (int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < total;
         x += int64_t(gridDim.x) * blockDim.x)
        out[x] = hash_entry(seed, scale, M, k0 + x / UM, x % UM);
}

// Sparse source, compressed by sorted tuple: T_0 row r is nonzero only if r is one of the
// listed tuples.  The rows are cleared by fill_zero first; this kernel writes the listed
// rows (one thread per listed tuple and mode).
template <typename C>
__global__ void __launch_bounds__(kThreads) fill_zero(C *__restrict__ out, int64_t count)
{
    for (int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < count;
         x += int64_t(gridDim.x) * blockDim.x)
        out[x] = from_d2<C>(make_double2(0.0, 0.0));
}

template <typename C, typename Acc>
__global__ void __launch_bounds__(kThreads)
psi_a_sparse(const double *__restrict__ vals, const int64_t *__restrict__ col_rank,
             const int64_t *__restrict__ col_ptr, const int32_t *__restrict__ row_k,
             int64_t ncols, const double2 *__restrict__ Psi, int64_t n, int64_t j0, int64_t J,
             int64_t Jpad, C *__restrict__ out)
{
    const int64_t total = ncols * Jpad;
    for (int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < total;
         x += int64_t(gridDim.x) * blockDim.x) {
        const int64_t c = x / Jpad, jj = x % Jpad;
        Acc re = 0, im = 0;
        if (jj < J) {
            const double2 *psi = Psi + (j0 + jj) * n;
            for (int64_t e = col_ptr[c]; e < col_ptr[c + 1]; ++e) {
                const Acc a = Acc(vals[e]);
                const double2 w = psi[row_k[e]];
                re += a * Acc(w.x);
                im += a * Acc(w.y);
            }
        }
        out[col_rank[c] * Jpad + jj] = from_d2<C>(make_double2(double(re), double(im)));
    }
}

// ---------------------------------------------------------------- lower-index chain
// Stage i: for sorted mode prefix p (length i-1, rank rp) and sorted state suffix s
// (length M-i, rank rs), and every t >= last(p):
//   T_i[rank(p U t)][rs][jj] = sum_a T_{i-1}[rp][rank(sort(a U s))][jj] Phi[a][t].
// LAST: i == M, writes C[jj][rank(p U t)] / M! as complex128 instead.
template <typename Cin, typename Cout, typename Acc, bool LAST>
__global__ void __launch_bounds__(kThreads)
stage_simt(const Cin *__restrict__ in, Cout *__restrict__ out, const double2 *__restrict__ Phi,
           int64_t n, int M, int i, int64_t U_prev, int64_t U_suf, int64_t U_in, int64_t J,
           int64_t Jpad, int64_t UM, double inv_fact, int64_t items)
{
    __shared__ int32_t p[kMaxOrder + 1], s[kMaxOrder + 1];
    extern __shared__ int64_t idx[];  // [n]
    for (int64_t item = blockIdx.x; item < items; item += gridDim.x) {
        const int64_t rp = item / U_suf, rs = item % U_suf;
        __syncthreads();
        if (threadIdx.x == 0) {
            colex_unrank(rp, i - 1, n, p);
            colex_unrank(rs, M - i, n, s);
        }
        __syncthreads();
        for (int64_t a = threadIdx.x; a < n; a += blockDim.x)
            idx[a] = colex_rank_insert(int32_t(a), s, M - i);
        __syncthreads();
        const int64_t last = (i > 1) ? p[i - 2] : 0;
        const int64_t base_p = (i > 1) ? colex_rank(p, i - 1) : 0;
        const int64_t nt = n - last;
        const Cin *src = in + rp * U_in * Jpad;
        for (int64_t x = threadIdx.x; x < nt * Jpad; x += blockDim.x) {
            const int64_t t = last + x / Jpad, jj = x % Jpad;
            Acc re = 0, im = 0;
            for (int64_t a = 0; a < n; ++a) {
                const double2 v = to_d2(src[idx[a] * Jpad + jj]);
                const double2 f = Phi[a * n + t];
                re += Acc(v.x) * Acc(f.x) - Acc(v.y) * Acc(f.y);
                im += Acc(v.x) * Acc(f.y) + Acc(v.y) * Acc(f.x);
            }
            // rank(p U t) with t >= last(p) appended at position i.
            const int64_t rpt = base_p + colex_term(t, i);
            if constexpr (LAST) {
                if (jj < J)
                    out[jj * UM + rpt] =
                        from_d2<Cout>(make_double2(double(re) * inv_fact, double(im) * inv_fact));
            } else {
                out[(rpt * U_suf + rs) * Jpad + jj] = from_d2<Cout>(make_double2(re, im));
            }
        }
    }
}

// ---------------------------------------------------------------- divisor and division
__global__ void __launch_bounds__(kThreads)
normal_form_simt(double2 *__restrict__ C, const double2 *__restrict__ lam, int64_t n, int M,
                 ModeMap mm, int64_t J, int64_t UM, double eps)
{
    const int64_t total = J * UM;
    int32_t t[kMaxOrder];
    for (int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < total;
         x += int64_t(gridDim.x) * blockDim.x) {
        const int64_t jj = x / UM, r = x % UM;
        colex_unrank(r, M, n, t);
        double2 acc = lam[t[0]];
        for (int l = 1; l < M; ++l) acc = add_fp64(acc, lam[t[l]]);
        const double2 d = divisor_fp64(acc, lam[mm.row[jj]], eps);
        C[x] = cdiv(C[x], d);
    }
}

// ---------------------------------------------------------------- reduction to P
// One thread per (mode j, state k): sequential sum over sorted tuples in colex order; the
// row of block mode jj is output mode mm.row[jj], and mm.conj[jj] gets the conjugate.
__global__ void __launch_bounds__(kThreads)
assemble_simt(const double2 *__restrict__ h, const double2 *__restrict__ Psi, int64_t n, int M,
              ModeMap mm, int64_t J, int64_t UM, double delta, double2 *__restrict__ P)
{
    const int64_t total = J * n;
    int32_t t[kMaxOrder];
    for (int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < total;
         x += int64_t(gridDim.x) * blockDim.x) {
        const int64_t jj = x / n, k = x % n;
        for (int l = 0; l < M; ++l) t[l] = 0;
        double sr = 0, si = 0;
        const double2 *hr = h + jj * UM;
        int64_t r = 0;
        do {
            double2 z = Psi[int64_t(t[0]) * n + k];
            z = make_double2(delta * z.x, delta * z.y);
            for (int l = 1; l < M; ++l) {
                const double2 w = Psi[int64_t(t[l]) * n + k];
                z = cmul(z, make_double2(delta * w.x, delta * w.y));
            }
            const double m = multiplicity(t, M);
            const double2 hz = cmul(hr[r], z);
            sr += m * hz.x;
            si += m * hz.y;
            ++r;
        } while (colex_next(t, M, n));
        double2 *dst = P + int64_t(mm.row[jj]) * n + k;
        *dst = make_double2(dst->x - sr, dst->y - si);
        if (mm.conj[jj] != kNoRow) {
            double2 *dc = P + int64_t(mm.conj[jj]) * n + k;
            *dc = make_double2(dc->x - sr, dc->y + si);
        }
    }
}

__global__ void __launch_bounds__(kThreads)
finalize_simt(const double2 *__restrict__ Psi, const double2 *__restrict__ Phi,
              const double2 *__restrict__ Psum, int64_t n, double delta, double2 *__restrict__ npf)
{
    const int64_t total = n * n;
    for (int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < total;
         x += int64_t(gridDim.x) * blockDim.x) {
        const int64_t k = x / n, i = x % n;
        const double2 w = Psi[i * n + k];
        double2 z = make_double2(delta * w.x, delta * w.y);
        if (Psum) z = add_fp64(z, Psum[i * n + k]);
        npf[x] = cmul(Phi[x], z);
    }
}

__global__ void __launch_bounds__(kThreads) zero_f64(double *x, int64_t count)
{
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
         i += int64_t(gridDim.x) * blockDim.x)
        x[i] = 0.0;
}

__global__ void __launch_bounds__(kThreads)
accumulate_f64(double *dst, const double *src, int64_t count, int first)
{
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
         i += int64_t(gridDim.x) * blockDim.x)
        dst[i] = first ? src[i] : dst[i] + src[i];
}

__global__ void __launch_bounds__(kThreads)
copy_rows_c128(double2 *dst, const double2 *src, int64_t n, int64_t j0, int64_t J)
{
    const int64_t total = J * n;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * blockDim.x)
        dst[j0 * n + i] = src[j0 * n + i];
}

unsigned grid_for(int64_t work, int64_t cap = 65536)
{
    int64_t g = (work + kThreads - 1) / kThreads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return unsigned(g);
}

}  // namespace

hipError_t launch_psi_a(const ChainArgs &a)
{
    const npf_plan_s &p = *a.plan;
    const int64_t UM = p.U[a.M];
    char *dst = a.ws + p.lay.buf[0];
    const double2 *Psi = reinterpret_cast<const double2 *>(a.U);
    const bool dense = a.A->kind == NPF_SRC_DENSE || a.A->kind == NPF_SRC_HASH;
    const int hashed = a.A->kind == NPF_SRC_HASH;
    if (dense && psi_a_mfma_supported(&p)) return launch_psi_a_mfma(a);
    if (dense) {
        if (p.prec == NPF_FP64)
            hipLaunchKernelGGL((psi_a_dense<double2, double>), dim3(grid_for(UM * p.Jpad)),
                               dim3(kThreads), 0, a.stream, a.A->values, Psi, p.n, UM, a.j0, a.J,
                               p.Jpad, reinterpret_cast<double2 *>(dst), hashed, a.A->seed,
                               a.A->scale, a.M);
        else
            hipLaunchKernelGGL((psi_a_dense<float2, double>), dim3(grid_for(UM * p.Jpad)),
                               dim3(kThreads), 0, a.stream, a.A->values, Psi, p.n, UM, a.j0, a.J,
                               p.Jpad, reinterpret_cast<float2 *>(dst), hashed, a.A->seed,
                               a.A->scale, a.M);
    } else {
        const int64_t total = a.A->ncols * p.Jpad;
        if (p.prec == NPF_FP64) {
            hipLaunchKernelGGL((fill_zero<double2>), dim3(grid_for(UM * p.Jpad)), dim3(kThreads),
                               0, a.stream, reinterpret_cast<double2 *>(dst), UM * p.Jpad);
            if (total > 0)
                hipLaunchKernelGGL((psi_a_sparse<double2, double>), dim3(grid_for(total)),
                                   dim3(kThreads), 0, a.stream, a.A->values, a.A->col_rank,
                                   a.A->col_ptr, a.A->row_k, a.A->ncols, Psi, p.n, a.j0, a.J,
                                   p.Jpad, reinterpret_cast<double2 *>(dst));
        } else {
            hipLaunchKernelGGL((fill_zero<float2>), dim3(grid_for(UM * p.Jpad)), dim3(kThreads),
                               0, a.stream, reinterpret_cast<float2 *>(dst), UM * p.Jpad);
            if (total > 0)
                hipLaunchKernelGGL((psi_a_sparse<float2, double>), dim3(grid_for(total)),
                                   dim3(kThreads), 0, a.stream, a.A->values, a.A->col_rank,
                                   a.A->col_ptr, a.A->row_k, a.A->ncols, Psi, p.n, a.j0, a.J,
                                   p.Jpad, reinterpret_cast<float2 *>(dst));
        }
    }
    return hipGetLastError();
}

hipError_t launch_hash_fill(double *out, uint64_t seed, double scale, int M, int64_t k0,
                            int64_t rows, int64_t UM, hipStream_t s)
{
    if (rows * UM > 0)
        hipLaunchKernelGGL(hash_fill, dim3(grid_for(rows * UM)), dim3(kThreads), 0, s, out, seed,
                           scale, M, k0, rows, UM);
    return hipGetLastError();
}

hipError_t launch_stage(const ChainArgs &a, int i)
{
    const npf_plan_s &p = *a.plan;
    const int M = a.M;
    const int64_t U_prev = p.U[i - 1], U_suf = p.U[M - i], U_in = p.U[M - i + 1];
    const int64_t items = U_prev * U_suf;
    const char *src = a.ws + p.lay.buf[(i - 1) % 2];
    char *dst = a.ws + p.lay.buf[i % 2];
    const double2 *Phi = reinterpret_cast<const double2 *>(a.V);
    const unsigned grid = unsigned(items < 262144 ? items : 262144);
    const size_t shm = sizeof(int64_t) * p.n;
    if (p.prec == NPF_FP64)
        hipLaunchKernelGGL((stage_simt<double2, double2, double, false>), dim3(grid),
                           dim3(kThreads), shm, a.stream, reinterpret_cast<const double2 *>(src),
                           reinterpret_cast<double2 *>(dst), Phi, p.n, M, i, U_prev, U_suf, U_in,
                           a.J, p.Jpad, p.U[M], 1.0, items);
    else
        hipLaunchKernelGGL((stage_simt<float2, float2, double, false>), dim3(grid), dim3(kThreads),
                           shm, a.stream, reinterpret_cast<const float2 *>(src),
                           reinterpret_cast<float2 *>(dst), Phi, p.n, M, i, U_prev, U_suf, U_in,
                           a.J, p.Jpad, p.U[M], 1.0, items);
    return hipGetLastError();
}

hipError_t launch_last_to_c(const ChainArgs &a, double *C_out)
{
    const npf_plan_s &p = *a.plan;
    const int M = a.M;
    const int i = M;
    const int64_t U_prev = p.U[M - 1], U_suf = 1, U_in = p.U[1];
    const int64_t items = U_prev;
    const char *src = a.ws + p.lay.buf[(M - 1) % 2];
    double fact = 1.0;
    for (int m = 2; m <= M; ++m) fact *= m;
    const double2 *Phi = reinterpret_cast<const double2 *>(a.V);
    const unsigned grid = unsigned(items < 262144 ? items : 262144);
    const size_t shm = sizeof(int64_t) * p.n;
    if (p.prec == NPF_FP64)
        hipLaunchKernelGGL((stage_simt<double2, double2, double, true>), dim3(grid),
                           dim3(kThreads), shm, a.stream, reinterpret_cast<const double2 *>(src),
                           reinterpret_cast<double2 *>(C_out), Phi, p.n, M, i, U_prev, U_suf,
                           U_in, a.J, p.Jpad, p.U[M], p.a_scale[M] / fact, items);
    else
        hipLaunchKernelGGL((stage_simt<float2, double2, double, true>), dim3(grid), dim3(kThreads),
                           shm, a.stream, reinterpret_cast<const float2 *>(src),
                           reinterpret_cast<double2 *>(C_out), Phi, p.n, M, i, U_prev, U_suf,
                           U_in, a.J, p.Jpad, p.U[M], p.a_scale[M] / fact, items);
    return hipGetLastError();
}

hipError_t launch_normal_form(const npf_plan_s *p, int M, int64_t j0, int64_t J,
                              const double *lam, double *C, hipStream_t s)
{
    const int64_t total = J * p->U[M];
    hipLaunchKernelGGL(normal_form_simt, dim3(grid_for(total)), dim3(kThreads), 0, s,
                       reinterpret_cast<double2 *>(C), reinterpret_cast<const double2 *>(lam),
                       p->n, M, mode_map(p, j0, J), J, p->U[M], p->prob.eps);
    return hipGetLastError();
}

hipError_t launch_assemble(const npf_plan_s *p, int M, int64_t j0, int64_t J, const double *h,
                           const double *U, double *P_acc, hipStream_t s)
{
    const int64_t total = J * p->n;
    hipLaunchKernelGGL(assemble_simt, dim3(grid_for(total)), dim3(kThreads), 0, s,
                       reinterpret_cast<const double2 *>(h), reinterpret_cast<const double2 *>(U),
                       p->n, M, mode_map(p, j0, J), J, p->U[M], p->prob.delta,
                       reinterpret_cast<double2 *>(P_acc));
    return hipGetLastError();
}

hipError_t launch_finalize(const npf_plan_s *p, const double *U, const double *V,
                           const double *P_sum, double *npf_out, hipStream_t s)
{
    hipLaunchKernelGGL(finalize_simt, dim3(grid_for(p->n * p->n)), dim3(kThreads), 0, s,
                       reinterpret_cast<const double2 *>(U), reinterpret_cast<const double2 *>(V),
                       reinterpret_cast<const double2 *>(P_sum), p->n, p->prob.delta,
                       reinterpret_cast<double2 *>(npf_out));
    return hipGetLastError();
}

hipError_t launch_zero(double *x, int64_t count, hipStream_t s)
{
    hipLaunchKernelGGL(zero_f64, dim3(grid_for(count)), dim3(kThreads), 0, s, x, count);
    return hipGetLastError();
}

hipError_t launch_accumulate(double *dst, const double *src, int64_t count, bool first,
                             hipStream_t s)
{
    hipLaunchKernelGGL(accumulate_f64, dim3(grid_for(count)), dim3(kThreads), 0, s, dst, src,
                       count, first ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_copy_rows(double *dst, const double *src, int64_t n, int64_t j0, int64_t J,
                            hipStream_t s)
{
    hipLaunchKernelGGL(copy_rows_c128, dim3(grid_for(J * n)), dim3(kThreads), 0, s,
                       reinterpret_cast<double2 *>(dst), reinterpret_cast<const double2 *>(src), n,
                       j0, J);
    return hipGetLastError();
}

}  // namespace npf
