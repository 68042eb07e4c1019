// Host-side planning: problem validation, the output-mode block size under the memory
// budget (the batch-size rule of Alg. 1), the workspace layout, and Alg. 1 itself.
#include <algorithm>
#include <cmath>
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

// Workspace layout for a block of Jpad output modes.
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
    const int64_t nparts = std::max<int64_t>(1, fused_max_slots(&p, Jpad));
    L.parts_bytes = nparts * Jpad * p.n * 16;
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
    const int64_t nparts = std::max<int64_t>(1, fused_max_slots(&p, Jpad));
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
        L.parts_bytes = nparts * Jpad * p.n * 16;
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
    if (q.n > 256) return fail(NPF_E_UNSUPPORTED, "n > 256 is not supported by the MFMA kernels");

    npf_plan_s *p = new (std::nothrow) npf_plan_s();
    if (!p) return fail(NPF_E_INVALID, "out of host memory");
    p->prob = q;
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
    // Block size over output modes: shrink the outermost (mode) dimension until the
    // working set fits the limit, then balance the blocks -- Alg. 1 steps 6-15 applied to
    // this path's working set.
    const int64_t full = round_up(q.n, 16);
    int64_t Jpad = full;
    if (q.block_modes > 0) Jpad = std::min(full, round_up(q.block_modes, 16));
    if (q.hbm_budget_bytes > 0) {
        while (Jpad >= 16 && make_layout(*p, Jpad).total > q.hbm_budget_bytes) Jpad -= 16;
        if (Jpad < 16) {
            delete p;
            return fail(NPF_E_BUDGET, "memory budget below the smallest block (16 modes)");
        }
    }
    p->n_blocks = (q.n + Jpad - 1) / Jpad;
    p->J = (q.n + p->n_blocks - 1) / p->n_blocks;
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
