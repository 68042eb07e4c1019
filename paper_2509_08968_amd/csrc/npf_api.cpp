// C ABI entry points: argument checks, block loops and kernel sequencing.
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "npf_internal.h"

using namespace npf;

namespace {

int check_hip(hipError_t e, const char *where)
{
    if (e == hipSuccess) return NPF_OK;
    return fail(NPF_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

}  // namespace

namespace npf {
int check_tensor(const npf_plan_s *p, const npf_tensor *A, int M)
{
    if (!A) return fail(NPF_E_INVALID, "null tensor descriptor");
    if (A->order != M) return fail(NPF_E_INVALID, "tensor order does not match the requested order");
    if (A->kind == NPF_SRC_DENSE) {
        if (!A->values) return fail(NPF_E_INVALID, "dense tensor without values");
        return NPF_OK;
    }
    if (A->kind == NPF_SRC_SPARSE) {
        if (!A->values || !A->col_rank || !A->col_ptr || !A->row_k)
            return fail(NPF_E_INVALID, "sparse tensor with a null array");
        if (A->ncols < 0 || A->ncols > p->U[M] || A->nnz < 0)
            return fail(NPF_E_INVALID, "sparse tensor sizes out of range");
        return NPF_OK;
    }
    if (A->kind == NPF_SRC_HASH) {
        if (p->n > 512 || p->U[M] >= (int64_t(1) << 40))
            return fail(NPF_E_UNSUPPORTED, "hash-generated tensors need n <= 512 and U_M < 2^40");
        if (!std::isfinite(A->scale)) return fail(NPF_E_INVALID, "hash tensor scale is not finite");
        return NPF_OK;
    }
    return fail(NPF_E_INVALID, "unknown tensor kind");
}
}  // namespace npf

namespace {

int check_order_block(const npf_plan_s *p, int32_t order, int64_t block)
{
    if (order < 2 || order > p->N) return fail(NPF_E_INVALID, "order outside [2, order_max]");
    if (block != NPF_ALL_BLOCKS && (block < 0 || block >= p->n_blocks))
        return fail(NPF_E_INVALID, "block index out of range");
    return NPF_OK;
}

// Blocks [b0, b1) selected by `block`.
void block_range(const npf_plan_s *p, int64_t block, int64_t &b0, int64_t &b1)
{
    if (block == NPF_ALL_BLOCKS) {
        b0 = 0;
        b1 = p->n_blocks;
    } else {
        b0 = block;
        b1 = block + 1;
    }
}

// Computed modes [j0, j0 + J) of block b (indices into the plan's computed-mode list).
void block_modes(const npf_plan_s *p, int64_t b, int64_t &j0, int64_t &J)
{
    j0 = b * p->J;
    J = p->nc - j0 < p->J ? p->nc - j0 : p->J;
}

std::string kname(int M, const char *what, int i = -1)
{
    std::string s = "o" + std::to_string(M) + "_" + what;
    if (i >= 0) s += std::to_string(i);
    return s;
}

// Per-row tables of the lower-indices-first route (once per order).
int run_rows(const npf_plan_s *p, int M, const npf_tensor *A, const void *V, void *ws, hipStream_t s)
{
    int rc;
    {
        Timed t(p, kname(M, "tucker_support"), s);
        rc = check_hip(launch_tucker_support(p, M, A, static_cast<char *>(ws), s),
                       "per-row support tables");
    }
    if (rc) return rc;
    Timed t(p, kname(M, "tucker_w"), s);
    return check_hip(launch_tucker_w(p, M, static_cast<const double *>(V), static_cast<char *>(ws), s),
                     "per-row lower-index contraction");
}

// T_{M-1} of the block [j0, j0 + J) in buffer (M-1) % 2: the upper-index contraction and
// the chain stages, or Psi applied to the per-row tables (tucker: run_rows done).
int run_chain(const npf_plan_s *p, int M, int64_t j0, int64_t J, const npf_tensor *A,
              const void *U, const void *V, void *ws, hipStream_t s, bool tucker = false)
{
    if (tucker) {
        Timed t(p, kname(M, "tucker_psi"), s);
        return check_hip(launch_tucker_psi(p, M, j0, J,
                                           psi_rows(p, static_cast<const double *>(U),
                                                    static_cast<const char *>(ws)),
                                           static_cast<char *>(ws), s),
                         "upper-index contraction of the per-row tables");
    }
    // The upper index runs over the computed modes: their staged Psi rows when the plan
    // selects modes.
    const double *Urows = psi_rows(p, static_cast<const double *>(U), static_cast<const char *>(ws));
    ChainArgs a{p, M, j0, J, A, Urows, static_cast<const double *>(V), static_cast<char *>(ws), s};
    int rc;
    {
        Timed t(p, kname(M, "psi_a"), s);
        rc = check_hip(launch_psi_a(a), "upper-index contraction");
    }
    const bool mfma = stage_mfma_supported(p);
    for (int i = 1; rc == NPF_OK && i < M; ++i) {
        Timed t(p, kname(M, "stage", i), s);
        rc = check_hip(mfma ? launch_stage_mfma(a, i) : launch_stage(a, i), "chain stage");
    }
    return rc;
}

int stage_operands(const npf_plan_s *p, const void *U, const void *V, const void *lam, void *ws,
                   hipStream_t s)
{
    Timed t(p, "prepare", s);
    return check_hip(launch_prepare(p, static_cast<const double *>(U),
                                    static_cast<const double *>(V),
                                    static_cast<const double *>(lam), static_cast<char *>(ws), s),
                     "operand staging");
}

}  // namespace

extern "C" int npf_modal_contract(npf_plan_t plan, int32_t order, int64_t block,
                                  const npf_tensor *A, const void *U, const void *V, void *ws,
                                  int64_t ws_bytes, void *C_out, void *stream)
{
    if (!plan) return fail(NPF_E_INVALID, "null plan");
    int rc = check_order_block(plan, order, block);
    if (rc) return rc;
    if ((rc = check_tensor(plan, A, order))) return rc;
    if (!U || !V || !ws || !C_out) return fail(NPF_E_INVALID, "null device pointer");
    if (ws_bytes < plan->lay.total) return fail(NPF_E_INVALID, "workspace smaller than planned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int64_t b0, b1;
    block_range(plan, block, b0, b1);
    const OrderLayout ol(plan, order);
    rc = stage_operands(plan, U, V, nullptr, ws, s);
    const bool tucker = tucker_supported(plan, A, order);
    if (!rc && tucker) rc = run_rows(plan, order, A, V, ws, s);
    for (int64_t b = b0; b < b1 && rc == NPF_OK; ++b) {
        int64_t j0, J;
        block_modes(plan, b, j0, J);
        const BlockShape shape(plan, J);
        rc = run_chain(plan, order, j0, J, A, U, V, ws, s, tucker);
        if (rc) break;
        double *dst = static_cast<double *>(C_out) + 2 * (j0 - b0 * plan->J) * plan->U[order];
        ChainArgs a{plan, order, j0, J, A, static_cast<const double *>(U),
                    static_cast<const double *>(V), static_cast<char *>(ws), s};
        rc = check_hip(launch_last_to_c(a, dst), "last contraction stage");
    }
    return rc;
}

extern "C" int npf_normal_form(npf_plan_t plan, int32_t order, int64_t block, const void *lambda,
                               void *C_inout, void *stream)
{
    if (!plan) return fail(NPF_E_INVALID, "null plan");
    int rc = check_order_block(plan, order, block);
    if (rc) return rc;
    if (!lambda || !C_inout) return fail(NPF_E_INVALID, "null device pointer");
    int64_t b0, b1;
    block_range(plan, block, b0, b1);
    int64_t j0a, Ja, j0b, Jb;
    block_modes(plan, b0, j0a, Ja);
    block_modes(plan, b1 - 1, j0b, Jb);
    return check_hip(launch_normal_form(plan, order, j0a, j0b + Jb - j0a,
                                        static_cast<const double *>(lambda),
                                        static_cast<double *>(C_inout),
                                        static_cast<hipStream_t>(stream)),
                     "normal form");
}

extern "C" int npf_assemble(npf_plan_t plan, int32_t order, int64_t block, const void *h,
                            const void *U, void *P_acc, void *stream)
{
    if (!plan) return fail(NPF_E_INVALID, "null plan");
    int rc = check_order_block(plan, order, block);
    if (rc) return rc;
    if (!h || !U || !P_acc) return fail(NPF_E_INVALID, "null device pointer");
    int64_t b0, b1;
    block_range(plan, block, b0, b1);
    int64_t j0a, Ja, j0b, Jb;
    block_modes(plan, b0, j0a, Ja);
    block_modes(plan, b1 - 1, j0b, Jb);
    return check_hip(launch_assemble(plan, order, j0a, j0b + Jb - j0a,
                                     static_cast<const double *>(h),
                                     static_cast<const double *>(U), static_cast<double *>(P_acc),
                                     static_cast<hipStream_t>(stream)),
                     "assemble");
}

extern "C" int npf_finalize(npf_plan_t plan, const void *U, const void *V, const void *P_sum,
                            void *npf_out, void *stream)
{
    if (!plan) return fail(NPF_E_INVALID, "null plan");
    if (!U || !V || !npf_out) return fail(NPF_E_INVALID, "null device pointer");
    return check_hip(launch_finalize(plan, static_cast<const double *>(U),
                                     static_cast<const double *>(V),
                                     static_cast<const double *>(P_sum),
                                     static_cast<double *>(npf_out),
                                     static_cast<hipStream_t>(stream)),
                     "finalize");
}

extern "C" int npf_hash_fill(int64_t n, int32_t order, uint64_t seed, double scale, int64_t k0,
                             int64_t k1, double *out, void *stream)
{
    if (n < 1 || n > 512) return fail(NPF_E_INVALID, "hash tensors need 1 <= n <= 512");
    if (order < 2 || order > NPF_MAX_ORDER) return fail(NPF_E_INVALID, "order outside [2, 6]");
    if (k0 < 0 || k1 > n || k0 > k1) return fail(NPF_E_INVALID, "row range outside [0, n]");
    const int64_t UM = binom(n + order - 1, order);
    if (UM >= (int64_t(1) << 40)) return fail(NPF_E_INVALID, "U_M >= 2^40");
    if (k1 == k0) return NPF_OK;
    if (!out) return fail(NPF_E_INVALID, "null output");
    return check_hip(launch_hash_fill(out, seed, scale, order, k0, k1 - k0, UM,
                                      static_cast<hipStream_t>(stream)),
                     "hash_fill");
}

namespace {

// The launch sequence of npf_run (eager).
struct SideSet;
int run_eager(npf_plan_t plan, const npf_tensor *A, const void *U, const void *V,
              const void *lambda, void *ws, void *P_out, void *npf_out, hipStream_t s,
              const SideSet *cs = nullptr);

// Side streams and events of the concurrent captures: one set per device, made on the
// first concurrent capture and kept for the life of the process, since the cached graphs
// captured from them outlive the plans.  Used only while capturing, under g_graph_mu.
struct SideSet {
    hipStream_t side[NPF_MAX_ORDER + 1] = {};   // side[M]: order M
    hipEvent_t ev_start = nullptr, ev_done[NPF_MAX_ORDER + 1] = {};
    bool ok = false;
};

// Graph cache: one instantiated graph per distinct argument set (problem, descriptors,
// pointers, stream), at most kMaxGraphs of them.  A plan is host metadata only: a later
// plan of the same problem replays the graph (the launches are a function of the key).
struct GraphKey {
    npf_problem prob;
    npf_tensor A[NPF_MAX_ORDER];
    const void *ptr[7];
    hipStream_t stream;
    ModeMap modes;               // the computed modes and their conjugate fills
};

bool same_key(const GraphKey &a, const GraphKey &b) { return std::memcmp(&a, &b, sizeof(a)) == 0; }

struct GraphEntry {
    GraphKey key;
    hipGraphExec_t exec;
    uint64_t used;
};

std::mutex g_graph_mu;
std::vector<GraphEntry> g_graphs;
uint64_t g_graph_clock = 0;
constexpr size_t kMaxGraphs = 16;
std::map<int, SideSet> g_side;

// The current device's side set (made on first use), or null if it cannot be made.
const SideSet *side_set()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    SideSet &S = g_side[dev];
    if (S.ok) return &S;
    for (int M = 2; M < NPF_MAX_ORDER; ++M)
        if (!S.side[M] && hipStreamCreateWithFlags(&S.side[M], hipStreamNonBlocking) != hipSuccess)
            return nullptr;
    for (int M = 2; M <= NPF_MAX_ORDER; ++M)
        if (!S.ev_done[M] && hipEventCreateWithFlags(&S.ev_done[M], hipEventDisableTiming) != hipSuccess)
            return nullptr;
    if (!S.ev_start && hipEventCreateWithFlags(&S.ev_start, hipEventDisableTiming) != hipSuccess)
        return nullptr;
    S.ok = true;
    return &S;
}

}  // namespace

namespace npf {
int run_eager_checked(npf_plan_t plan, const npf_tensor *A, const void *U, const void *V,
                      const void *lambda, void *ws, int64_t ws_bytes, void *P_out, void *npf_out,
                      hipStream_t s)
{
    if (!plan) return fail(NPF_E_INVALID, "null plan");
    if (!A || !U || !V || !lambda || !ws) return fail(NPF_E_INVALID, "null argument");
    if (ws_bytes < plan->lay.total) return fail(NPF_E_INVALID, "workspace smaller than planned");
    int rc = NPF_OK;
    for (int M = 2; M <= plan->N; ++M)
        if ((rc = check_tensor(plan, &A[M - 2], M))) return rc;
    return run_eager(plan, A, U, V, lambda, ws, P_out, npf_out, s);
}
}  // namespace npf

extern "C" int npf_run(npf_plan_t plan, const npf_tensor *A, const void *U, const void *V,
                       const void *lambda, void *ws, int64_t ws_bytes, void *P_out, void *npf_out,
                       void *stream)
{
    if (!plan) return fail(NPF_E_INVALID, "null plan");
    if (!A || !U || !V || !lambda || !ws) return fail(NPF_E_INVALID, "null argument");
    if (ws_bytes < plan->lay.total) return fail(NPF_E_INVALID, "workspace smaller than planned");
    int rc = NPF_OK;
    for (int M = 2; M <= plan->N; ++M)
        if ((rc = check_tensor(plan, &A[M - 2], M))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    bool graph = !(plan->prob.flags & NPF_FLAG_NO_GRAPH) && !plan->prof.on && s != nullptr;
    if (graph) {
        hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &st) != hipSuccess || st != hipStreamCaptureStatusNone)
            graph = false;
    }
    if (!graph) return run_eager(plan, A, U, V, lambda, ws, P_out, npf_out, s);

    GraphKey key;
    std::memset(&key, 0, sizeof(key));
    key.prob = plan->prob;
    for (int M = 2; M <= plan->N; ++M) key.A[M - 2] = A[M - 2];
    const void *ptrs[7] = {U, V, lambda, ws, P_out, npf_out, reinterpret_cast<const void *>(ws_bytes)};
    std::memcpy(key.ptr, ptrs, sizeof(ptrs));
    key.stream = s;
    key.modes = mode_map(plan, 0, plan->nc);
    std::lock_guard<std::mutex> lock(g_graph_mu);
    for (auto &e : g_graphs)
        if (same_key(e.key, key)) {
            e.used = ++g_graph_clock;
            return check_hip(hipGraphLaunch(e.exec, s), "graph launch");
        }
    // A full cache runs new argument sets eagerly: cached graphs are not destroyed while the
    // process runs (a host fault was seen when evicting them under many distinct problems).
    if (g_graphs.size() >= kMaxGraphs) return run_eager(plan, A, U, V, lambda, ws, P_out, npf_out, s);
    const SideSet *cs = plan->concurrent ? side_set() : nullptr;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return run_eager(plan, A, U, V, lambda, ws, P_out, npf_out, s);
    rc = run_eager(plan, A, U, V, lambda, ws, P_out, npf_out, s, cs);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(s, &g);
    if (rc != NPF_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (ec != hipSuccess || !g) return check_hip(ec != hipSuccess ? ec : hipErrorUnknown, "graph capture");
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return check_hip(ei, "graph instantiate");
    g_graphs.push_back({key, exec, ++g_graph_clock});
    return check_hip(hipGraphLaunch(exec, s), "graph launch");
}

namespace {

int run_eager(npf_plan_t plan, const npf_tensor *A, const void *U, const void *V,
              const void *lambda, void *ws, void *P_out, void *npf_out, hipStream_t s,
              const SideSet *cs)
{
    const bool concurrent = cs != nullptr;
    // Concurrent (captured runs of single-block plans with several orders): after the operand
    // staging, order M < N runs its chain, last stage and partial sums on side stream M while
    // order N runs on the caller's stream; the partial sums follow the order of M.
    int rc = NPF_OK;
    char *w = static_cast<char *>(ws);
    const int64_t nn = plan->n * plan->n;
    // Operand staging first on the caller's stream; concurrent runs fork after it (a
    // dependency of the chains on staging work queued on another stream was seen to hold the
    // longest chain behind the other orders' kernels).
    rc = stage_operands(plan, U, V, lambda, ws, s);
    if (!rc && concurrent) rc = check_hip(hipEventRecord(cs->ev_start, s), "fork");
    auto reduce = [&](int M, int64_t j0, int64_t J, hipStream_t st) {
        const OrderLayout ol(plan, M);
        double *PM = P_out ? static_cast<double *>(P_out) + 2 * (M - 2) * nn
                           : reinterpret_cast<double *>(w + plan->lay.pm);
        double *psum = reinterpret_cast<double *>(w + plan->lay.psum);
        // The last order's partial sums also write the NPF (Alg. 2 step 20).
        const NpfOut fin{static_cast<const double *>(U), static_cast<const double *>(V),
                         static_cast<double *>(npf_out)};
        Timed t(plan, kname(M, "reduce"), st);
        return check_hip(launch_reduce_parts(plan, M, j0, J, PM, psum, M == 2, w, st,
                                             (M == plan->N && npf_out) ? &fin : nullptr),
                         "partial sums");
    };
    // Concurrent runs enqueue the highest order (the longest chain, on the caller's stream)
    // first, so that its launches are not queued behind the shorter orders'.
    for (int q = 0; q <= plan->N - 2 && rc == NPF_OK; ++q) {
        const int M = concurrent ? plan->N - q : 2 + q;
        const bool on_side = concurrent && M < plan->N;
        const hipStream_t sm = on_side ? cs->side[M] : s;
        if (on_side && (rc = check_hip(hipStreamWaitEvent(sm, cs->ev_start, 0), "fork"))) break;
        const OrderLayout ol(plan, M);
        const bool tucker = tucker_supported(plan, &A[M - 2], M);
        if (tucker) rc = run_rows(plan, M, &A[M - 2], V, ws, sm);
        for (int64_t b = 0; b < plan->n_blocks && rc == NPF_OK; ++b) {
            int64_t j0, J;
            block_modes(plan, b, j0, J);
            const BlockShape shape(plan, J);
            rc = run_chain(plan, M, j0, J, &A[M - 2], U, V, ws, sm, tucker);
            if (rc) break;
            {
                Timed t(plan, kname(M, "fused"), sm);
                rc = check_hip(launch_fused_last(plan, M, j0, J,
                                                 static_cast<const double *>(lambda), w, sm),
                               "fused last stage");
            }
            if (!rc && !concurrent) rc = reduce(M, j0, J, s);
        }
    }
    // Partial sums of a concurrent run: order M < N on its side stream right after its last
    // stage and after order M - 1's sums (the NPF sum is accumulated in order), the highest
    // order's on the caller's stream after order N - 1's -- so only the last one follows the
    // longest chain.
    if (concurrent)
        for (int M = 2; M <= plan->N && rc == NPF_OK; ++M) {
            const hipStream_t sm = M < plan->N ? cs->side[M] : s;
            if (M > 2) rc = check_hip(hipStreamWaitEvent(sm, cs->ev_done[M - 1], 0), "join");
            if (!rc) rc = reduce(M, 0, plan->nc, sm);
            if (!rc && M < plan->N) rc = check_hip(hipEventRecord(cs->ev_done[M], sm), "join");
        }
    return rc;
}

}  // namespace

extern "C" int npf_run_interaction(npf_plan_t plan, const npf_tensor *A, const void *U,
                                   const void *V, const void *lambda, void *ws, int64_t ws_bytes,
                                   void *P_out, void *npf_out, void *inpf_out, void *stream)
{
    if (!plan) return fail(NPF_E_INVALID, "null plan");
    if (!inpf_out) return fail(NPF_E_INVALID, "null interaction output");
    if (plan->n_out != plan->n)
        return fail(NPF_E_UNSUPPORTED,
                    "interaction factors need every mode's P row (zeta* of eq. (9)): no mode subset");
    // First pass: P_M of every order and the NPF (npf_run checks the remaining arguments).
    int rc = npf_run(plan, A, U, V, lambda, ws, ws_bytes, P_out, npf_out, stream);
    if (rc) return rc;
    // Second pass: the reduction factor becomes zeta* = delta Psi + sum_M P_M, and every
    // order's last contraction and reduction run again on it (the chain is recomputed: a
    // later block or order may have overwritten it).
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    {
        Timed t(plan, "prepare_zeta_star", s);
        rc = check_hip(launch_prepare(plan, static_cast<const double *>(U),
                                      static_cast<const double *>(V),
                                      static_cast<const double *>(lambda), w, s,
                                      reinterpret_cast<const double *>(w + plan->lay.psum)),
                       "zeta* staging");
    }
    const int64_t nn = plan->n * plan->n;
    for (int M = 2; M <= plan->N && rc == NPF_OK; ++M) {
        const OrderLayout ol(plan, M);
        const bool tucker = tucker_supported(plan, &A[M - 2], M);
        if (tucker) rc = run_rows(plan, M, &A[M - 2], V, ws, s);
        double *out = static_cast<double *>(inpf_out) + 2 * (M - 2) * nn;
        for (int64_t b = 0; b < plan->n_blocks && rc == NPF_OK; ++b) {
            int64_t j0, J;
            block_modes(plan, b, j0, J);
            const BlockShape shape(plan, J);
            rc = run_chain(plan, M, j0, J, &A[M - 2], U, V, ws, s, tucker);
            if (rc) break;
            {
                Timed t(plan, kname(M, "fused_star"), s);
                rc = check_hip(launch_fused_last(plan, M, j0, J,
                                                 static_cast<const double *>(lambda), w, s),
                               "fused last stage (zeta*)");
            }
            if (rc) break;
            // Phi for the factors of eq. (8); no NPF output in this pass.
            const NpfOut fin{static_cast<const double *>(U), static_cast<const double *>(V),
                             nullptr};
            Timed t(plan, kname(M, "reduce_star"), s);
            rc = check_hip(launch_reduce_parts(plan, M, j0, J, nullptr, nullptr, false, w, s,
                                               &fin, out),
                           "interaction factors");
        }
    }
    return rc;
}
