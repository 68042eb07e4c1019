/*
 * CPU FP64 oracle for the NPF hot path -- TEST INFRASTRUCTURE ONLY (see npf_oracle.h).
 *
 * Plain loops in double / double complex, built with -O2 -ffp-contract=off and no
 * fast-math.  Every function names the passage of the paper it follows:
 *   eq. (4)      normal-form coefficient h = (Psi A Phi..Phi) / (lam_r + .. + lam_v - lam_i)
 *   eq. (7)      z(0) = zeta - h2 zeta zeta - .. - hN zeta..zeta, zeta = delta Psi[:, k]
 *   Alg. 2       steps 1-4 contraction, 5-9 divisor and clamp, 11 division,
 *                12-19 Khatri-Rao power of Psi and reduction, 20 assembly.
 *   eqs. (8)-(9) interaction factors pNM[k,i] = Phi[k,i] sum_t h_M[i,t] prod_l zeta*_k[t_l],
 *                with zeta*_k = delta Psi[:,k] + sum_M P_M[:,k] (= z(0) of eq. (7)): the same
 *                reduction with zeta* in place of zeta (npfo_sym_z, npfo_full_z: P of zeta*).
 * Readings where the paper is silent (all listed in the design notes):
 *   - A_M is the derivative tensor, so the Taylor coefficient is A_M / M! (Alg. 2 step 4).
 *   - The divisor is summed over the sorted tuple left to right, then lam_j subtracted,
 *     so that near a resonance every implementation rounds it the same way.
 *   - The clamp of step 9 is applied literally (|D| < eps -> D = eps, real), decided as
 *     re*re + im*im < eps*eps in double without fused multiply-add.
 *   - "Phi . (Psi + sum PsiN)" in step 20 is the entrywise product aligned as
 *     (state k, mode i), which is the only reading that reduces to the linear
 *     participation factor phi_ki psi_ik of eq. (7) when h = 0.
 *   - The permutation of step 16 does not change the result, because the Khatri-Rao
 *     power of step 18 is symmetric in its tuple; the sum runs over t in [n]^M directly.
 */
#include "npf_oracle.h"

#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int64_t npfo_binom(int64_t a, int64_t b)
{
    if (b < 0 || a < 0 || b > a) return 0;
    if (b > a - b) b = a - b;
    int64_t r = 1;
    for (int64_t i = 1; i <= b; ++i) r = r * (a - b + i) / i;   /* exact at every step */
    return r;
}

int64_t npfo_rank(const int32_t *t, int m)
{
    int64_t r = 0;
    for (int i = 0; i < m; ++i) r += npfo_binom((int64_t)t[i] + i, i + 1);
    return r;
}

/* Sorted m-tuple with colex rank r. */
static void unrank(int64_t r, int m, int64_t n, int32_t *t)
{
    for (int i = m; i >= 1; --i) {
        int64_t x = 0;
        while (x + 1 < n && npfo_binom(x + 1 + i - 1, i) <= r) ++x;
        t[i - 1] = (int32_t)x;
        r -= npfo_binom(x + i - 1, i);
    }
}

/* Next sorted m-tuple over [0, n) in colex order; returns 0 after the last one. */
static int next_sorted(int32_t *t, int m, int64_t n)
{
    for (int i = 0; i < m; ++i) {
        int64_t cap = (i + 1 < m) ? t[i + 1] : n - 1;
        if (t[i] < cap) {
            t[i] += 1;
            for (int l = 0; l < i; ++l) t[l] = 0;
            return 1;
        }
    }
    return 0;
}

static double factorial(int m)
{
    double f = 1.0;
    for (int i = 2; i <= m; ++i) f *= (double)i;
    return f;
}

/* Alg. 2 steps 5-9 for one sorted tuple s (ascending) and output mode j. */
static npfo_c divisor(const npfo_c *lam, const int32_t *s, int M, int64_t j, double eps)
{
    npfo_c acc = lam[s[0]];
    for (int i = 1; i < M; ++i) acc = acc + lam[s[i]];
    npfo_c d = acc - lam[j];
    double re = creal(d), im = cimag(d);
    double mag2 = re * re;
    mag2 = mag2 + im * im;
    if (mag2 < eps * eps) d = eps;
    return d;
}

/* Number of distinct orderings of a sorted tuple, M! / prod(count_v!). */
static double multiplicity(const int32_t *s, int M)
{
    double m = factorial(M);
    int run = 1;
    for (int i = 1; i <= M; ++i) {
        if (i < M && s[i] == s[i - 1]) {
            ++run;
        } else {
            m /= factorial(run);
            run = 1;
        }
    }
    return m;
}

static void sort_small(int32_t *s, int m)
{
    for (int i = 1; i < m; ++i) {
        int32_t v = s[i];
        int l = i - 1;
        while (l >= 0 && s[l] > v) { s[l + 1] = s[l]; --l; }
        s[l + 1] = v;
    }
}

/* ------------------------------------------------------------------ full tensors */
static int full_impl(int64_t n, int M, const npfo_c *lam, const npfo_c *Phi, const npfo_c *Psi,
                     const double *A_full, double eps, double delta, const npfo_c *Z,
                     npfo_c *C_full, npfo_c *h_full, npfo_c *P);

int npfo_full(int64_t n, int M, const npfo_c *lam, const npfo_c *Phi, const npfo_c *Psi,
              const double *A_full, double eps, double delta,
              npfo_c *C_full, npfo_c *h_full, npfo_c *P)
{
    return full_impl(n, M, lam, Phi, Psi, A_full, eps, delta, NULL, C_full, h_full, P);
}

int npfo_full_z(int64_t n, int M, const npfo_c *lam, const npfo_c *Phi, const npfo_c *Psi,
                const double *A_full, double eps, const npfo_c *Z, npfo_c *P)
{
    if (!Z) return -1;
    return full_impl(n, M, lam, Phi, Psi, A_full, eps, 1.0, Z, NULL, NULL, P);
}

/* The reduction's factor for mode t and kicked state k: delta Psi[t, k] (eq. (7)), or the
 * given Z[t, k] (the corrected zeta* of eq. (9) for the interaction factors of eq. (8)). */
static npfo_c zeta_at(const npfo_c *Z, const npfo_c *Psi, double delta, int64_t n, int64_t t,
                      int64_t k)
{
    return Z ? Z[t * n + k] : delta * Psi[t * n + k];
}

static int full_impl(int64_t n, int M, const npfo_c *lam, const npfo_c *Phi, const npfo_c *Psi,
                     const double *A_full, double eps, double delta, const npfo_c *Z,
                     npfo_c *C_full, npfo_c *h_full, npfo_c *P)
{
    if (n < 1 || M < 2 || M > 8 || !lam || !Phi || !Psi || !A_full || !(eps > 0.0)) return -1;
    int64_t nm = 1;
    for (int i = 0; i < M; ++i) nm *= n;
    const int64_t total = n * nm;
    npfo_c *T = malloc(sizeof(npfo_c) * total);
    npfo_c *W = malloc(sizeof(npfo_c) * total);
    npfo_c *C = C_full ? C_full : malloc(sizeof(npfo_c) * total);
    npfo_c *h = h_full ? h_full : malloc(sizeof(npfo_c) * total);
    if (!T || !W || !C || !h) return -1;

    /* Steps 1-3: T <- AN, then contract lower index p (1..M) with Phi:
     * T[k, t_1..t_{p-1}, a, ..] -> W[k, t_1..t_{p-1}, t_p, ..] = sum_a T[..a..] Phi[a, t_p]. */
    for (int64_t x = 0; x < total; ++x) T[x] = A_full[x];
    for (int p = 1; p <= M; ++p) {
        int64_t inner = 1;
        for (int i = p; i < M; ++i) inner *= n;
        const int64_t outer = total / (n * inner);
        for (int64_t o = 0; o < outer; ++o)
            for (int64_t tp = 0; tp < n; ++tp)
                for (int64_t in = 0; in < inner; ++in) {
                    npfo_c s = 0;
                    for (int64_t a = 0; a < n; ++a)
                        s = s + T[(o * n + a) * inner + in] * Phi[a * n + tp];
                    W[(o * n + tp) * inner + in] = s;
                }
        npfo_c *sw = T; T = W; W = sw;
    }
    /* Step 4: C[j, t] = sum_k Psi[j, k] T[k, t] / M!. */
    const double fact = factorial(M);
    for (int64_t j = 0; j < n; ++j)
        for (int64_t t = 0; t < nm; ++t) {
            npfo_c s = 0;
            for (int64_t k = 0; k < n; ++k) s = s + Psi[j * n + k] * T[k * nm + t];
            C[j * nm + t] = s / fact;
        }
    /* Steps 5-11: divisor over the sorted tuple, clamp, division. */
    int32_t digits[8], srt[8];
    for (int64_t j = 0; j < n; ++j)
        for (int64_t t = 0; t < nm; ++t) {
            int64_t rem = t;
            for (int i = M - 1; i >= 0; --i) { digits[i] = (int32_t)(rem % n); rem /= n; }
            memcpy(srt, digits, sizeof(int32_t) * M);
            sort_small(srt, M);
            npfo_c d = divisor(lam, srt, M, j, eps);
            h[j * nm + t] = C[j * nm + t] / d;
        }
    /* Steps 12-19: P[j, k] = - sum_{t in [n]^M} h[j, t] prod_i (delta Psi[t_i, k]). */
    if (P) {
        for (int64_t j = 0; j < n; ++j)
            for (int64_t k = 0; k < n; ++k) {
                npfo_c s = 0;
                for (int64_t t = 0; t < nm; ++t) {
                    int64_t rem = t;
                    for (int i = M - 1; i >= 0; --i) { digits[i] = (int32_t)(rem % n); rem /= n; }
                    npfo_c z = zeta_at(Z, Psi, delta, n, digits[0], k);
                    for (int i = 1; i < M; ++i) z = z * zeta_at(Z, Psi, delta, n, digits[i], k);
                    s = s + h[j * nm + t] * z;
                }
                P[j * n + k] = -s;
            }
    }
    free(T);
    free(W);
    if (!C_full) free(C);
    if (!h_full) free(h);
    return 0;
}

/* ------------------------------------------------------------------ packed symmetric */
/* Colex rank of sort(a U s) for a sorted m-tuple s. */
static int64_t rank_insert(int32_t a, const int32_t *s, int m)
{
    int32_t merged[9];
    int w = 0, placed = 0;
    for (int i = 0; i < m; ++i) {
        if (!placed && a <= s[i]) { merged[w++] = a; placed = 1; }
        merged[w++] = s[i];
    }
    if (!placed) merged[w++] = a;
    return npfo_rank(merged, m + 1);
}

/* Hash-generated tensor entry (order M, state k, colex rank r): SplitMix64 output number
 * (M << 49 | k << 40 | r) for the seed, its four 16-bit fields summed to S, and
 * ((S - 131070) * 2^-16 * sqrt(3)) * scale, the two roundings in that order. */
static uint64_t splitmix64_at(uint64_t seed, uint64_t idx)
{
    uint64_t z = seed + (idx + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double npfo_hash_value(uint64_t seed, double scale, int M, int64_t k, int64_t r)
{
    const uint64_t idx = ((uint64_t)M << 49) | ((uint64_t)k << 40) | (uint64_t)r;
    const uint64_t w = splitmix64_at(seed, idx);
    int64_t S = 0;
    for (int q = 0; q < 4; ++q) S += (int64_t)((w >> (16 * q)) & 0xFFFFu);
    const double x = (double)(S - 131070) * (1.0 / 65536.0);
    const double y = x * 1.7320508075688772;
    return y * scale;
}

static int sym_impl(int64_t n, int M, const npfo_c *lam, const npfo_c *Phi, const npfo_c *Psi,
                    const double *A_packed, int hashed, uint64_t seed, double scale,
                    double eps, double delta, const npfo_c *Z, const int64_t *modes,
                    int64_t n_modes, npfo_c *C_sym, npfo_c *h_sym, npfo_c *P_rows, int nthreads);

int npfo_sym(int64_t n, int M, const npfo_c *lam, const npfo_c *Phi, const npfo_c *Psi,
             const double *A_packed, double eps, double delta,
             const int64_t *modes, int64_t n_modes,
             npfo_c *C_sym, npfo_c *h_sym, npfo_c *P_rows, int nthreads)
{
    if (!A_packed) return -1;
    return sym_impl(n, M, lam, Phi, Psi, A_packed, 0, 0, 0.0, eps, delta, NULL, modes, n_modes,
                    C_sym, h_sym, P_rows, nthreads);
}

int npfo_sym_hash(int64_t n, int M, const npfo_c *lam, const npfo_c *Phi, const npfo_c *Psi,
                  uint64_t seed, double scale, double eps, double delta,
                  const int64_t *modes, int64_t n_modes,
                  npfo_c *C_sym, npfo_c *h_sym, npfo_c *P_rows, int nthreads)
{
    if (n > 512) return -1;
    return sym_impl(n, M, lam, Phi, Psi, NULL, 1, seed, scale, eps, delta, NULL, modes, n_modes,
                    C_sym, h_sym, P_rows, nthreads);
}

int npfo_sym_z(int64_t n, int M, const npfo_c *lam, const npfo_c *Phi, const npfo_c *Psi,
               const double *A_packed, double eps, const npfo_c *Z, const int64_t *modes,
               int64_t n_modes, npfo_c *P_rows, int nthreads)
{
    if (!A_packed || !Z) return -1;
    return sym_impl(n, M, lam, Phi, Psi, A_packed, 0, 0, 0.0, eps, 1.0, Z, modes, n_modes, NULL,
                    NULL, P_rows, nthreads);
}

static int sym_impl(int64_t n, int M, const npfo_c *lam, const npfo_c *Phi, const npfo_c *Psi,
                    const double *A_packed, int hashed, uint64_t seed, double scale,
                    double eps, double delta, const npfo_c *Z, const int64_t *modes,
                    int64_t n_modes, npfo_c *C_sym, npfo_c *h_sym, npfo_c *P_rows, int nthreads)
{
    if (n < 1 || M < 2 || M > 8 || !lam || !Phi || !Psi || (!A_packed && !hashed) || !modes ||
        n_modes < 0 || !(eps > 0.0))
        return -1;
    for (int64_t q = 0; q < n_modes; ++q)
        if (modes[q] < 0 || modes[q] >= n) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    int64_t Ucount[10];
    for (int m = 0; m <= M; ++m) Ucount[m] = npfo_binom(n + m - 1, m);
    const int64_t UM = Ucount[M];
    int64_t maxsz = 0;
    for (int i = 0; i <= M; ++i) {
        int64_t sz = Ucount[i] * Ucount[M - i];
        if (sz > maxsz) maxsz = sz;
    }
    npfo_c *Tprev = malloc(sizeof(npfo_c) * maxsz);
    npfo_c *Tnext = malloc(sizeof(npfo_c) * maxsz);
    npfo_c *h = malloc(sizeof(npfo_c) * UM);
    if (!Tprev || !Tnext || !h) return -1;
    const double fact = factorial(M);

    for (int64_t q = 0; q < n_modes; ++q) {
        const int64_t j = modes[q];
        /* Upper index first: G[r] = sum_k Psi[j, k] A_M[k, r] over sorted state tuples. */
#pragma omp parallel for schedule(static)
        for (int64_t r = 0; r < UM; ++r) {
            npfo_c s = 0;
            for (int64_t k = 0; k < n; ++k) {
                const double a = hashed ? npfo_hash_value(seed, scale, M, k, r) : A_packed[k * UM + r];
                s = s + Psi[j * n + k] * a;
            }
            Tprev[r] = s;
        }
        /* Lower indices one by one (Alg. 2 steps 2-3).  Stage i maps
         * T_{i-1}[p][sort(a U s)] (p: sorted modes, length i-1; s: sorted states, length
         * M-i) to T_i[p U t][s] = sum_a T_{i-1}[p][sort(a U s)] Phi[a, t] for t >= last(p). */
        for (int i = 1; i <= M; ++i) {
            const int64_t np_ = Ucount[i - 1], ns = Ucount[M - i], nin = Ucount[M - i + 1];
            const int64_t items = np_ * ns;
#pragma omp parallel
            {
                int64_t *idx = malloc(sizeof(int64_t) * n);
                npfo_c *acc = malloc(sizeof(npfo_c) * n);
                int32_t p[9], s[9], pt[9];
#pragma omp for schedule(dynamic, 16)
                for (int64_t it = 0; it < items; ++it) {
                    const int64_t rp = it / ns, rs = it % ns;
                    unrank(rp, i - 1, n, p);
                    unrank(rs, M - i, n, s);
                    const int64_t last = (i > 1) ? p[i - 2] : 0;
                    for (int64_t a = 0; a < n; ++a) idx[a] = rank_insert((int32_t)a, s, M - i);
                    for (int64_t t = 0; t < n; ++t) acc[t] = 0;
                    for (int64_t a = 0; a < n; ++a) {
                        const npfo_c x = Tprev[rp * nin + idx[a]];
                        if (x == 0) continue;   /* adding 0 * Phi leaves every sum unchanged */
                        for (int64_t t = last; t < n; ++t) acc[t] = acc[t] + x * Phi[a * n + t];
                    }
                    for (int l = 0; l < i - 1; ++l) pt[l] = p[l];
                    for (int64_t t = last; t < n; ++t) {
                        pt[i - 1] = (int32_t)t;
                        Tnext[npfo_rank(pt, i) * ns + rs] = acc[t];
                    }
                }
                free(idx);
                free(acc);
            }
            npfo_c *sw = Tprev; Tprev = Tnext; Tnext = sw;
        }
        /* Step 4 (1/M!), steps 5-9 (divisor, clamp) and step 11 (division). */
        const int64_t chunk = 4096, nchunks = (UM + chunk - 1) / chunk;
#pragma omp parallel
        {
            int32_t t[9];
#pragma omp for schedule(static)
            for (int64_t ch = 0; ch < nchunks; ++ch) {
                const int64_t r0 = ch * chunk, r1 = (r0 + chunk < UM) ? r0 + chunk : UM;
                unrank(r0, M, n, t);
                for (int64_t r = r0; r < r1; ++r) {
                    const npfo_c c = Tprev[r] / fact;
                    const npfo_c hv = c / divisor(lam, t, M, j, eps);
                    h[r] = hv;
                    if (C_sym) C_sym[q * UM + r] = c;
                    if (h_sym) h_sym[q * UM + r] = hv;
                    next_sorted(t, M, n);
                }
            }
        }
        /* Steps 12-19 over sorted tuples: each sorted t stands for multiplicity(t)
         * orderings with the same h (h is symmetric in t) and the same product. */
        if (P_rows) {
#pragma omp parallel
            {
                int32_t t[9];
#pragma omp for schedule(static)
                for (int64_t k = 0; k < n; ++k) {
                    for (int l = 0; l < M; ++l) t[l] = 0;
                    npfo_c s = 0;
                    int64_t r = 0;
                    do {
                        npfo_c z = zeta_at(Z, Psi, delta, n, t[0], k);
                        for (int l = 1; l < M; ++l) z = z * zeta_at(Z, Psi, delta, n, t[l], k);
                        s = s + multiplicity(t, M) * (h[r] * z);
                        ++r;
                    } while (next_sorted(t, M, n));
                    P_rows[q * n + k] = -s;
                }
            }
        }
    }
    free(Tprev);
    free(Tnext);
    free(h);
    return 0;
}

int npfo_assemble(int64_t n, const npfo_c *Phi, const npfo_c *Psi, double delta,
                  const npfo_c *Psum, npfo_c *npf)
{
    if (n < 1 || !Phi || !Psi || !npf) return -1;
    for (int64_t k = 0; k < n; ++k)
        for (int64_t i = 0; i < n; ++i) {
            npfo_c z = delta * Psi[i * n + k];
            if (Psum) z = z + Psum[i * n + k];
            npf[k * n + i] = Phi[k * n + i] * z;
        }
    return 0;
}

/* ------------------------------------------------------------------ derivative tensors
 * The M-th derivative tensor of a polynomial vector field at the expansion point x* (the
 * tensors the numerical Taylor expansion of Alg. 1 produces from the model): for each term
 * c * prod_v x_v^{e_v} of equation k, x = x* + y gives
 *   c * prod_v sum_{j_v} binom(e_v, j_v) x*_v^{e_v - j_v} y_v^{j_v},
 * whose part of total degree M in y, sum_v j_v = M, contributes
 *   c * prod_v binom(e_v, j_v) x*_v^{e_v - j_v} * prod_v j_v!
 * to the derivative d^M f_k / dy_{a_1} .. dy_{a_M} for the sorted tuple a holding each
 * variable v j_v times (differentiating prod_v y_v^{j_v} once by each of those variables
 * leaves prod_v j_v!).  Terms: eq[q], coef[q], var[q*maxdeg + i] (the monomial's variables
 * with repetition, padded with -1).  out[k*U + rank(a)], zeroed first. */
int npfo_poly_tensor(int64_t n, int M, int64_t n_terms, const int32_t *eq, const double *coef,
                     const int32_t *var, int maxdeg, const double *x_eq, double *out)
{
    if (n < 1 || M < 1 || M > 8 || maxdeg < 0 || maxdeg > 8 || (n_terms > 0 && (!eq || !coef || !var))
        || !out)
        return -1;
    const int64_t U = npfo_binom(n + M - 1, M);
    for (int64_t x = 0; x < n * U; ++x) out[x] = 0.0;
    for (int64_t q = 0; q < n_terms; ++q) {
        /* distinct variables of the monomial and their exponents */
        int32_t v[8], e[8];
        int nv = 0;
        for (int i = 0; i < maxdeg; ++i) {
            const int32_t a = var[q * maxdeg + i];
            if (a < 0) continue;
            if (a >= n) return -1;
            int f = -1;
            for (int l = 0; l < nv; ++l) if (v[l] == a) f = l;
            if (f < 0) { v[nv] = a; e[nv] = 1; ++nv; } else e[f] += 1;
        }
        if (eq[q] < 0 || eq[q] >= n) return -1;
        /* every split j_l <= e_l with sum_l j_l = M */
        int32_t j[8] = {0};
        for (;;) {
            int tot = 0;
            for (int l = 0; l < nv; ++l) tot += j[l];
            if (tot == M) {
                double w = coef[q];
                int32_t t[8];
                int m = 0;
                for (int l = 0; l < nv; ++l) {
                    w *= (double)npfo_binom(e[l], j[l]) * factorial(j[l]);
                    const double xs = x_eq ? x_eq[v[l]] : 0.0;
                    for (int r = 0; r < e[l] - j[l]; ++r) w *= xs;
                    for (int r = 0; r < j[l]; ++r) t[m++] = v[l];
                }
                sort_small(t, M);
                out[(int64_t)eq[q] * U + npfo_rank(t, M)] += w;
            }
            int l = 0;                          /* next split (odometer over j_l <= e_l) */
            while (l < nv && j[l] == e[l]) { j[l] = 0; ++l; }
            if (l == nv) break;
            j[l] += 1;
        }
    }
    return 0;
}
