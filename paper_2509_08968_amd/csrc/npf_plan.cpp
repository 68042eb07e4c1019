// Host-side planning: problem validation, the output-mode block size under the memory
// budget (the batch-size rule of Alg. 1), the workspace layout, and Alg. 1 itself.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <new>

#include "npf_internal.h"

namespace npf {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int code, const std::string &msg)
{
    set_error(msg);
    return code;
}

int64_t binom(int64_t a, int64_t b)
{
    if (b < 0 || a < 0 || b > a) return 0;
    if (b > a - b) b = a - b;
    int64_t r = 1;
    for (int64_t i = 1; i <= b; ++i) r = r * (a - b + i) / i;
    return r;
}

static int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Partial-P slots x block width of the widest layout any block of at most Jpad modes uses
// (a narrower last block may write more slots of fewer modes).
static int64_t parts_elems(const npf_plan_s &p, int64_t Jpad)
{
    int64_t e = 0;
    for (int64_t w = 16; w <= Jpad; w += 16)
        e = std::max(e, std::max<int64_t>(1, fused_max_slots(&p, w)) * w);
    return e;
}

// Workspace layout for blocks of at most Jpad output modes.
static Layout make_layout(const npf_plan_s &p, int64_t Jpad)
{
    Layout L;
    int64_t per[2] = {0, 0};
    for (int M = 2; M <= p.N; ++M)
        for (int i = 0; i < M; ++i) {
            const int64_t sz = p.U[i] * p.U[M - i] * Jpad * p.esz;
            per[i % 2] = std::max(per[i % 2], sz);
        }
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        const int64_t at = off;
        off += round_up(std::max<int64_t>(bytes, 0), 256);
        return at;
    };
    L.buf_bytes[0] = per[0];
    L.buf_bytes[1] = per[1];
    L.buf[0] = take(per[0]);
    L.buf[1] = take(per[1]);
    L.ttab = take(p.tt.total * 8);
    L.psum = take(p.n * p.n * 16);
    L.pm = take(p.n * p.n * 16);
    L.phi_bytes = p.npad * p.npad * 16 * 4;
    L.phi = take(L.phi_bytes);
    if (p.select) L.msel = take(p.nc * (p.n + 1) * 16);
    L.parts_bytes = parts_elems(p, Jpad) * p.n * 16;
    L.parts = take(L.parts_bytes);
    const int smax = p.prob.support_max;
    if (smax >= 1 && smax <= kTuckerMaxSupport && p.N >= 2) {
        const int Mt = std::min(p.N, 3);          // the route serves orders 2 and 3
        L.tk.over = take(p.n * 4);
        L.tk.S = take(p.n * smax * 4);
        L.tk.cnt = take(p.n * 4);
        L.tk.inv = take(p.n * p.n * 4);
        L.tk.invcnt = take(p.n * 4);
        L.tk.D = take(p.n * binom(smax + Mt - 1, Mt) * 8);
        if (Mt == 3) L.tk.Y = take(p.n * smax * p.n * smax * 16);
        L.tk.W = take(p.U[Mt - 1] * p.n * smax * 16);
    }
    L.total = off;
    return L;
}

// Layout with a region per order for concurrent orders: common parts once, then for each
// order M its chain buffers, partials, P scratch and per-row tables.  ord[M] are complete
// layouts (the common offsets repeated); the returned layout's total covers all of them.
static Layout make_split_layout(const npf_plan_s &p, int64_t Jpad, Layout *ord)
{
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        const int64_t at = off;
        off += round_up(std::max<int64_t>(bytes, 0), 256);
        return at;
    };
    Layout C;
    C.ttab = take(p.tt.total * 8);
    C.psum = take(p.n * p.n * 16);
    C.phi_bytes = p.npad * p.npad * 16 * 4;
    C.phi = take(C.phi_bytes);
    if (p.select) C.msel = take(p.nc * (p.n + 1) * 16);
    const int smax = p.prob.support_max;
    for (int M = 2; M <= p.N; ++M) {
        Layout L = C;
        int64_t per[2] = {0, 0};
        for (int i = 0; i < M; ++i) per[i % 2] = std::max(per[i % 2], p.U[i] * p.U[M - i] * Jpad * p.esz);
        L.buf_bytes[0] = per[0];
        L.buf_bytes[1] = per[1];
        L.buf[0] = take(per[0]);
        L.buf[1] = take(per[1]);
        L.pm = take(p.n * p.n * 16);
        L.parts_bytes = parts_elems(p, Jpad) * p.n * 16;
        L.parts = take(L.parts_bytes);
        if (tucker_route(&p, M)) {
            L.tk.over = take(p.n * 4);
            L.tk.S = take(p.n * smax * 4);
            L.tk.cnt = take(p.n * 4);
            L.tk.inv = take(p.n * p.n * 4);
            L.tk.invcnt = take(p.n * 4);
            L.tk.D = take(p.n * binom(smax + M - 1, M) * 8);
            if (M == 3) L.tk.Y = take(p.n * smax * p.n * smax * 16);
            L.tk.W = take(p.U[M - 1] * p.n * smax * 16);
        }
        ord[M] = L;
    }
    for (int M = 2; M <= p.N; ++M) ord[M].total = off;
    Layout R = ord[p.N];
    R.total = off;
    return R;
}

// Output modes, conjugate pairs and the preconditions with host copies (Alg. 2 needs
// Psi Phi = I; the pairing of conj_of must hold for the filled modes to be right).
static int check_modes(const npf_problem &q, std::vector<int32_t> &cm, std::vector<int32_t> &cj,
                       int64_t &n_out)
{
    const int64_t n = q.n;
    std::vector<char> out(size_t(n), q.n_modes == 0 ? 1 : 0);
    if (q.n_modes < 0 || q.n_modes > n) return fail(NPF_E_INVALID, "n_modes outside [0, n]");
    if (q.n_modes > 0) {
        if (!q.modes) return fail(NPF_E_INVALID, "n_modes > 0 with a null mode list");
        for (int64_t i = 0; i < q.n_modes; ++i) {
            const int64_t j = q.modes[i];
            if (j < 0 || j >= n) return fail(NPF_E_INVALID, "output mode outside [0, n)");
            if (out[size_t(j)]) return fail(NPF_E_INVALID, "output mode listed twice");
            out[size_t(j)] = 1;
        }
    }
    if (q.conj_of)
        for (int64_t i = 0; i < n; ++i) {
            const int64_t c = q.conj_of[i];
            if (c < 0 || c >= n || q.conj_of[c] != i)
                return fail(NPF_E_INVALID, "conj_of is not an involution on [0, n)");
        }
    cm.clear();
    cj.clear();
    n_out = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (!out[size_t(i)]) continue;
        ++n_out;
        const int64_t c = q.conj_of ? q.conj_of[i] : i;
        if (c != i && out[size_t(c)]) {
            if (c < i) continue;                       // filled from its partner c
            cm.push_back(int32_t(i));
            cj.push_back(int32_t(c));
        } else {
            cm.push_back(int32_t(i));
            cj.push_back(-1);
        }
    }
    return NPF_OK;
}

static int check_host_copies(const npf_problem &q)
{
    const double tol = q.check_tol > 0.0 ? q.check_tol : 1e-8;
    const int64_t n = q.n;
    using cd = std::complex<double>;
    const cd *U = static_cast<const cd *>(q.host_U);
    const cd *V = static_cast<const cd *>(q.host_V);
    const cd *lam = static_cast<const cd *>(q.host_lambda);
    if (U && V)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j) {
                cd s = 0.0;
                for (int64_t k = 0; k < n; ++k) s += U[i * n + k] * V[k * n + j];
                if (std::abs(s - (i == j ? cd(1.0) : cd(0.0))) > tol)
                    return fail(NPF_E_INVALID, "Psi Phi differs from the identity by more than check_tol");
            }
    if (!q.conj_of) return NPF_OK;
    auto maxabs = [](const cd *x, int64_t count) {
        double m = 0.0;
        for (int64_t e = 0; e < count; ++e) m = std::max(m, std::abs(x[e]));
        return m > 0.0 ? m : 1.0;
    };
    const double sl = lam ? maxabs(lam, n) : 1.0, su = U ? maxabs(U, n * n) : 1.0,
                 sv = V ? maxabs(V, n * n) : 1.0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t c = q.conj_of[i];
        if (lam && std::abs(lam[c] - std::conj(lam[i])) > tol * sl)
            return fail(NPF_E_INVALID, "conj_of pairs eigenvalues that are not conjugate");
        for (int64_t k = 0; k < n; ++k) {
            if (V && std::abs(V[k * n + c] - std::conj(V[k * n + i])) > tol * sv)
                return fail(NPF_E_INVALID, "conj_of pairs right eigenvectors that are not conjugate");
            if (U && std::abs(U[c * n + k] - std::conj(U[i * n + k])) > tol * su)
                return fail(NPF_E_INVALID, "conj_of pairs left eigenvectors that are not conjugate");
        }
    }
    return NPF_OK;
}

ModeMap mode_map(const npf_plan_s *p, int64_t c0, int64_t J)
{
    ModeMap m;
    for (int q = 0; q < kMaxModes; ++q) {
        const int64_t c = c0 + q;
        const bool in = q < J && c < p->nc;
        m.row[q] = in ? uint16_t(p->cm[size_t(c)]) : kNoRow;
        m.conj[q] = (in && p->cj[size_t(c)] >= 0) ? uint16_t(p->cj[size_t(c)]) : kNoRow;
    }
    return m;
}

const double *psi_rows(const npf_plan_s *p, const double *U, const char *ws)
{
    return p->select ? reinterpret_cast<const double *>(ws + p->lay.msel) : U;
}

const double *lam_rows(const npf_plan_s *p, const double *lam, const char *ws)
{
    return p->select ? reinterpret_cast<const double *>(ws + p->lay.msel) + 2 * p->nc * p->n : lam;
}

}  // namespace npf

using namespace npf;

extern "C" int npf_plan_create(const npf_problem *problem, npf_plan_t *plan_out)
{
    if (!problem || !plan_out) return fail(NPF_E_INVALID, "npf_plan_create: null argument");
    *plan_out = nullptr;
    const npf_problem &q = *problem;
    if (q.n < 1) return fail(NPF_E_INVALID, "n must be >= 1");
    if (q.order_max < 2 || q.order_max > NPF_MAX_ORDER)
        return fail(NPF_E_INVALID, "order_max must be in [2, NPF_MAX_ORDER]");
    if (q.precision != NPF_FP64 && q.precision != NPF_FP32 && q.precision != NPF_BF16X3)
        return fail(NPF_E_INVALID, "unknown precision");
    if (!(q.eps > 0.0) || !std::isfinite(q.eps)) return fail(NPF_E_INVALID, "eps must be > 0");
    if (!(q.tau >= 0.0) || !std::isfinite(q.tau)) return fail(NPF_E_INVALID, "tau must be >= 0");
    if (!std::isfinite(q.delta)) return fail(NPF_E_INVALID, "delta must be finite");
    if (q.hbm_budget_bytes < 0 || q.block_modes < 0)
        return fail(NPF_E_INVALID, "negative budget or block size");
    if (q.support_max < 0) return fail(NPF_E_INVALID, "negative support bound");
    if (q.a_convention != NPF_A_DERIVATIVE && q.a_convention != NPF_A_TAYLOR)
        return fail(NPF_E_INVALID, "unknown derivative-tensor convention");
    if (!(q.check_tol >= 0.0) || !std::isfinite(q.check_tol))
        return fail(NPF_E_INVALID, "check_tol must be >= 0");
    if (q.n > 512) return fail(NPF_E_UNSUPPORTED, "n > 512 is not supported (tuple entries are 9 bits)");
    if (q.n > 256 && q.precision == NPF_BF16X3)
        return fail(NPF_E_UNSUPPORTED, "split-BF16 plans serve n <= 256; use FP32 or FP64 above");
    // The mixed paths store C once per sorted tuple in FP32, and every ordering of the tuple
    // reuses that one rounding; beyond order 4 (m(t) up to 120 orderings) the coherent error
    // exceeds the 1e-6 bound of these paths, so orders 5 and 6 are served in FP64 only.
    if (q.precision != NPF_FP64 && q.order_max > kMixedMaxOrder)
        return fail(NPF_E_UNSUPPORTED, "FP32 and split-BF16 plans serve orders up to 4; use FP64 for orders 5-6");

    std::vector<int32_t> cm, cj;
    int64_t n_out = 0;
    int rc = check_modes(q, cm, cj, n_out);
    if (rc) return rc;
    if ((q.host_U || q.host_V || q.host_lambda) && (rc = check_host_copies(q))) return rc;

    npf_plan_s *p = new (std::nothrow) npf_plan_s();
    if (!p) return fail(NPF_E_INVALID, "out of host memory");
    p->prob = q;
    // The plan keeps its own copies; no caller pointer outlives the call.
    p->prob.modes = nullptr;
    p->prob.conj_of = nullptr;
    p->prob.host_U = p->prob.host_V = p->prob.host_lambda = nullptr;
    p->cm = std::move(cm);
    p->cj = std::move(cj);
    p->nc = int64_t(p->cm.size());
    p->n_out = n_out;
    p->select = p->nc != q.n;
    for (int64_t c = 0; c < p->nc && !p->select; ++c) p->select = p->cm[size_t(c)] != c || p->cj[size_t(c)] >= 0;
    double fact = 1.0;
    for (int M = 2; M <= NPF_MAX_ORDER; ++M) {
        fact *= M;
        p->a_scale[M] = q.a_convention == NPF_A_TAYLOR ? fact : 1.0;
    }
    p->n = q.n;
    p->N = q.order_max;
    p->prec = q.precision;
    p->esz = (q.precision == NPF_FP64) ? 16 : 8;
    p->npad = round_up(q.n, 32);
    for (int m = 0; m <= p->N; ++m) {
        p->U[m] = binom(q.n + m - 1, m);
        if (p->U[m] <= 0 || p->U[m] > (int64_t(1) << 40)) {
            delete p;
            return fail(NPF_E_UNSUPPORTED, "tuple count overflows the supported range");
        }
    }
    p->tt.maxlen = p->N - 1;
    for (int m = 1; m <= p->N - 1; ++m) {
        p->tt.count[m] = p->U[m];
        p->tt.off[m] = p->tt.total;
        p->tt.total += p->U[m];
    }
    // Block size over the computed modes: shrink the outermost (mode) dimension until the
    // working set fits the limit, then balance the blocks -- Alg. 1 steps 6-15 applied to
    // this path's working set.
    const int64_t nc = std::max<int64_t>(p->nc, 1);
    const int64_t full = round_up(nc, 16);
    int64_t Jpad = full;
    if (q.block_modes > 0) Jpad = std::min(full, round_up(q.block_modes, 16));
    if (q.hbm_budget_bytes > 0) {
        while (Jpad >= 16 && make_layout(*p, Jpad).total > q.hbm_budget_bytes) Jpad -= 16;
        if (Jpad < 16) {
            delete p;
            return fail(NPF_E_BUDGET, "memory budget below the smallest block (16 modes)");
        }
    }
    // Balanced blocks, or full blocks of Jpad modes and a narrower last one when that pads
    // fewer modes (100 modes under a 32-mode limit: 32 + 32 + 32 + 16 rather than 4 x 32).
    p->n_blocks = (nc + Jpad - 1) / Jpad;
    const int64_t J_bal = (nc + p->n_blocks - 1) / p->n_blocks;
    const int64_t padded_bal = p->n_blocks * round_up(J_bal, 16);
    const int64_t padded_full = (p->n_blocks - 1) * Jpad + round_up(nc - (p->n_blocks - 1) * Jpad, 16);
    p->J = padded_full < padded_bal ? Jpad : J_bal;
    p->Jpad = round_up(p->J, 16);
    p->lay = make_layout(*p, p->Jpad);
    for (int M = 0; M <= NPF_MAX_ORDER; ++M) p->ord[M] = p->lay;
    if (!(q.flags & NPF_FLAG_SERIAL_ORDERS) && p->n_blocks == 1 && p->N >= 3) {
        Layout ord[NPF_MAX_ORDER + 1];
        const Layout split = make_split_layout(*p, p->Jpad, ord);
        if (q.hbm_budget_bytes == 0 || split.total <= q.hbm_budget_bytes) {
            p->concurrent = true;
            p->lay = split;
            for (int M = 2; M <= p->N; ++M) p->ord[M] = ord[M];
        }
    }
    *plan_out = p;
    return NPF_OK;
}

extern "C" int npf_plan_info(npf_plan_t plan, npf_plan_report *r)
{
    if (!plan || !r) return fail(NPF_E_INVALID, "npf_plan_info: null argument");
    std::memset(r, 0, sizeof(*r));
    r->n = plan->n;
    r->order_max = plan->N;
    r->precision = plan->prec;
    r->workspace_bytes = plan->lay.total;
    r->block_modes = plan->J;
    r->n_blocks = plan->n_blocks;
    int64_t entries = 0;
    for (int m = 0; m <= plan->N; ++m) {
        r->unique_tuples[m] = plan->U[m];
        if (m >= 2) entries += plan->n * plan->U[m];
    }
    r->modal_entries = entries;
    r->output_modes = plan->n_out;
    r->computed_modes = plan->nc;
    return NPF_OK;
}

extern "C" int npf_plan_modes(npf_plan_t plan, int64_t *computed, int64_t *filled)
{
    if (!plan) return fail(NPF_E_INVALID, "npf_plan_modes: null plan");
    for (int64_t c = 0; c < plan->nc; ++c) {
        if (computed) computed[c] = plan->cm[size_t(c)];
        if (filled) filled[c] = plan->cj[size_t(c)];
    }
    return NPF_OK;
}

extern "C" void npf_plan_destroy(npf_plan_t plan) { delete plan; }

// Alg. 1 steps 1-15: the full tensor has n_dim dimensions of extent n_s; while its size
// exceeds the limit, drop the outermost dimension and either batch it one index at a time
// (when the remaining part alone is still too large) or in batches of
// E_max = floor(limit / size of the remaining part).
extern "C" int64_t npf_alg1_batches(int32_t n_dim, int64_t n_s, double m_limit_gb,
                                    int32_t bytes_per_entry, int64_t *BC, int64_t *max_batch,
                                    double *total_gb, double *batch_gb)
{
    if (n_dim < 1 || n_dim > 64 || n_s < 1 || !(m_limit_gb > 0.0) || bytes_per_entry < 1 ||
        !BC || !max_batch)
        return -1;
    const double gib = 1024.0 * 1024.0 * 1024.0;
    for (int d = 0; d < n_dim; ++d) {
        BC[d] = 1;
        max_batch[d] = n_s;
    }
    double tc = std::pow(double(n_s), double(n_dim));
    double m = tc * bytes_per_entry / gib;
    if (total_gb) *total_gb = m;
    int nd = n_dim;
    while (m > m_limit_gb && nd > 0) {
        nd -= 1;
        const double mf = std::pow(double(n_s), double(nd)) * bytes_per_entry / gib;
        if (mf > m_limit_gb) {
            BC[nd] = n_s;
            max_batch[nd] = 1;
        } else {
            const int64_t emax = int64_t(std::floor(m_limit_gb / mf));
            BC[nd] = (n_s + emax - 1) / emax;
            max_batch[nd] = std::min(emax, n_s);
        }
        m = mf;
    }
    int64_t nb = 1;
    double per = double(bytes_per_entry) / gib;
    for (int d = 0; d < n_dim; ++d) {
        nb *= BC[d];
        per *= double(max_batch[d]);
    }
    if (batch_gb) *batch_gb = per;
    return nb;
}

extern "C" const char *npf_error_string(int code)
{
    switch (code) {
    case NPF_OK: return "ok";
    case NPF_E_INVALID: return "invalid argument";
    case NPF_E_BUDGET: return "memory budget too small";
    case NPF_E_DEVICE: return "device error";
    case NPF_E_UNSUPPORTED: return "unsupported";
    default: return "unknown error";
    }
}

extern "C" const char *npf_last_error(void) { return g_last_error.c_str(); }
