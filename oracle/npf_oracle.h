/*
 * CPU FP64 oracle for the nonlinear-participation-factor (NPF) hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or calls this
 * code; only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
 * do.  It shares no source with the HIP path.
 *
 * What it computes (all in double / double complex, order M >= 2 at a time):
 *   C[j,t]  = (1/M!) sum_k Psi[j,k] sum_{a in [n]^M} A_M[k,a] prod_i Phi[a_i, t_i]
 *             -- eq. (4) numerator, Alg. 2 steps 1-4 (A_M is a derivative tensor).
 *   D[j,t]  = (lam[s_1] + ... + lam[s_M]) - lam[j],  s = t sorted ascending, summed left
 *             to right; if |D|^2 < eps^2 then D := eps           -- Alg. 2 steps 5-9.
 *   h[j,t]  = C[j,t] / D[j,t]                                     -- Alg. 2 step 11, eq. (4).
 *   P_M[j,k] = - sum_{t in [n]^M} h[j,t] prod_i (delta Psi[t_i,k]) -- eq. (7), steps 12-19.
 *   NPF[k,i] = Phi[k,i] (delta Psi[i,k] + sum_M P_M[i,k])          -- eq. (7), step 20.
 *
 * Array conventions (row-major, complex = interleaved re/im = C99 double _Complex):
 *   lam[n]; Phi[a*n + i] = Phi[state a, mode i]; Psi[i*n + k] = Psi[mode i, state k].
 *   A_full[k*n^M + (a_1 n^{M-1} + ... + a_M)]   full derivative tensor (real).
 *   A_packed[k*U + rank(t)], U = binom(n+M-1, M), t sorted, colex
 *       rank(t) = sum_{i=1..M} binom(t_i + i - 1, i).
 *   P[j*n + k]; NPF[k*n + i].
 * Functions return 0 on success, -1 on invalid arguments (nothing written).
 */
#ifndef NPF_ORACLE_H
#define NPF_ORACLE_H

#include <stdint.h>
#include <complex.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef double _Complex npfo_c;

/* binom(a, b) as int64 (0 when b < 0 or b > a). */
int64_t npfo_binom(int64_t a, int64_t b);
/* Colex rank of a sorted m-tuple. */
int64_t npfo_rank(const int32_t *t, int m);

/* Literal Alg. 2 on full tensors: successive mode products with Phi on every lower
 * index (steps 1-3), the upper index with Psi and 1/M! (step 4), the divisor (5-9),
 * the division (11) and the reduction over all t in [n]^M (12-19).
 * Outputs (any may be NULL): C_full, h_full [n * n^M] complex, P [n*n] complex.
 * Memory ~ 2 n^{M+1} complex: for small n only. */
int npfo_full(int64_t n, int M, const npfo_c *lam, const npfo_c *Phi, const npfo_c *Psi,
              const double *A_full, double eps, double delta,
              npfo_c *C_full, npfo_c *h_full, npfo_c *P);

/* The same quantities from packed symmetric storage, one output mode at a time:
 * G = Psi[j,:] A_M (upper index first), then the lower indices one by one with Phi,
 * keeping only sorted mode tuples (T_i is symmetric in its contracted and in its
 * remaining indices).  modes[n_modes] selects output modes j.
 * Outputs (any may be NULL): C_sym, h_sym [n_modes * U] complex (row = selected mode,
 * column = colex rank of the sorted mode tuple), P_rows [n_modes * n] complex.
 * nthreads <= 0 uses the OpenMP default. */
int npfo_sym(int64_t n, int M, const npfo_c *lam, const npfo_c *Phi, const npfo_c *Psi,
             const double *A_packed, double eps, double delta,
             const int64_t *modes, int64_t n_modes,
             npfo_c *C_sym, npfo_c *h_sym, npfo_c *P_rows, int nthreads);

/* The reduction of Alg. 2 steps 12-19 with a given factor matrix in place of zeta = delta Psi:
 * P_rows[q*n + k] = - sum_{t in [n]^M} h[modes[q], t] prod_i Z[t_i*n + k] (sym: packed
 * tensors, per selected mode) and P[j*n + k] likewise for every j (full: full tensors, small
 * n).  With Z[a*n + k] = zeta*_k[a] (eq. (9): delta Psi[a,k] + sum_M P_M[a,k]), -P is the
 * contraction of h_M with M factors zeta* whose Hadamard product with Phi gives the
 * interaction participation factors of eq. (8). */
int npfo_sym_z(int64_t n, int M, const npfo_c *lam, const npfo_c *Phi, const npfo_c *Psi,
               const double *A_packed, double eps, const npfo_c *Z, const int64_t *modes,
               int64_t n_modes, npfo_c *P_rows, int nthreads);
int npfo_full_z(int64_t n, int M, const npfo_c *lam, const npfo_c *Phi, const npfo_c *Psi,
                const double *A_full, double eps, const npfo_c *Z, npfo_c *P);

/* Entry A_M[k, r] of a hash-generated tensor (seed, scale): SplitMix64 (Steele, Lea and
 * Flood 2014) output number (M << 49 | k << 40 | r) from the seed; S = sum of its four
 * 16-bit fields; value = ((S - 131070) * 2^-16 * sqrt(3)) * scale (Irwin-Hall sum of
 * four uniforms, mean 0, variance about scale^2). */
double npfo_hash_value(uint64_t seed, double scale, int M, int64_t k, int64_t r);

/* npfo_sym with A_M generated entry by entry by npfo_hash_value (n <= 512). */
int npfo_sym_hash(int64_t n, int M, const npfo_c *lam, const npfo_c *Phi, const npfo_c *Psi,
                  uint64_t seed, double scale, double eps, double delta,
                  const int64_t *modes, int64_t n_modes,
                  npfo_c *C_sym, npfo_c *h_sym, npfo_c *P_rows, int nthreads);

/* NPF[k*n+i] = Phi[k,i] * (delta Psi[i,k] + Psum[i*n+k]); Psum may be NULL (linear PF). */
int npfo_assemble(int64_t n, const npfo_c *Phi, const npfo_c *Psi, double delta,
                  const npfo_c *Psum, npfo_c *npf);

/* The M-th derivative tensor, packed over sorted tuples, of the polynomial vector field
 * f_k(x) = sum_{terms q of equation k} coef[q] prod_i x_{var[q*maxdeg + i]} (variables with
 * repetition, -1 = none) at the expansion point x_eq (NULL = 0): out[k*U_M + rank(a)] =
 * d^M f_k / dx_{a_1} .. dx_{a_M} at x_eq, from the binomial expansion of every monomial --
 * the tensors Alg. 1 obtains by numerical Taylor expansion of the model. */
int npfo_poly_tensor(int64_t n, int M, int64_t n_terms, const int32_t *eq, const double *coef,
                     const int32_t *var, int maxdeg, const double *x_eq, double *out);

#ifdef __cplusplus
}
#endif
#endif
