// Batched operating points: many systems of uneven n through the whole hot path in one
// call.  Systems are grouped in waves whose summed workspace fits the budget (the memory
// limit of Alg. 1 applied across systems).  Within a wave, each chain stage and the fused
// last stage of an order run as one launch per padded size over all systems of that size:
// the launch's workgroups are shared out in proportion to each system's work and every
// system reads its own argument record, so small systems do not leave the GPU idle.  The
// light per-system steps (operand staging, the upper-index contraction, the partial sums,
// the assembly) are launched per system.  On a non-NULL stream the whole sequence is
// captured once per argument set and replayed.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "npf_bf3.h"

using namespace npf;

namespace {

constexpr int64_t kTargets[] = {256, 512, 1024, 2048, 4096};   // autotuner candidates

// One launch over several systems of the same padded size.
struct Shared {
    int wave = 0;
    int kind = 0;              // 0: chain stage i of order M; 1: fused last stage of order M
    int npad = 0, M = 0, i = 0;
    int gy = 1;
    std::vector<int> sys;      // batch indices of the systems
    std::vector<int64_t> cap;  // most workgroups per system
    std::vector<double> work;  // work estimate per system
    int64_t target = 1024;     // workgroups per launch
    double flops = 0;          // algorithmic flops of the launch
    float ms = 0;              // measured duration (npf_batch_time)
    std::vector<int32_t> first;
    int64_t args_off = 0, first_off = 0;   // byte offsets in the argument table
};

struct Sys {
    npf_plan_s *plan = nullptr;
    int wave = 0;
    int64_t off = 0;           // workspace offset within the wave region
};

struct GraphEntry {
    std::vector<uintptr_t> key;
    hipGraphExec_t exec = nullptr;
    void *table = nullptr;     // pinned host copy of the argument table this graph uploads
    hipEvent_t done = nullptr; // recorded after every launch of the graph
    uint64_t used = 0;
};

// Graphs kept per batch; further argument sets run eagerly (a cached graph is destroyed only
// with the batch, or when the autotuner changes the launches, and only after its last
// launch has completed).
constexpr size_t kMaxBatchGraphs = 4;

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Orders that take the lower-indices-first route (sparse tensors with a support bound).
bool planned_tucker(const npf_plan_s *p, int M) { return tucker_route(p, M); }

}  // namespace

struct npf_batch_s {
    std::vector<Sys> sys;
    std::vector<std::vector<int>> waves;
    int Nmax = 0;
    int64_t wave_bytes = 0, table_bytes = 0, ws_bytes = 0, entries = 0, launches = 0;
    std::vector<Shared> shared;
    void *table = nullptr;          // pinned staging for eager runs
    hipEvent_t table_done = nullptr;
    bool table_pending = false;
    std::vector<GraphEntry> graphs;
    uint64_t clock = 0;
    std::mutex mu;
    ~npf_batch_s();
};

namespace {

// Destroys the cached graphs.  Each one's last launch may still be running (or waiting on
// its stream); the pinned table its copy node reads and the executable are released only
// after the event recorded behind that launch has completed.
void free_graphs(npf_batch_s *b)
{
    for (auto &g : b->graphs) {
        if (g.done) {
            (void)hipEventSynchronize(g.done);
            (void)hipEventDestroy(g.done);
        }
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.table) (void)hipHostFree(g.table);
    }
    b->graphs.clear();
}

int launch_graph(GraphEntry &g, hipStream_t st)
{
    hipError_t e = hipGraphLaunch(g.exec, st);
    if (e == hipSuccess) e = hipEventRecord(g.done, st);
    if (e == hipSuccess) return NPF_OK;
    return fail(NPF_E_DEVICE, std::string("graph launch: ") + hipGetErrorString(e));
}

// Workgroups per system of a shared launch, in proportion to the work, at least one and at
// most the system's cap.
void share_out(Shared &L)
{
    double W = 0;
    for (double w : L.work) W += w;
    L.first.assign(L.sys.size() + 1, 0);
    for (size_t q = 0; q < L.sys.size(); ++q) {
        int64_t g = W > 0 ? int64_t(std::llround(double(L.target) * L.work[q] / W)) : 1;
        g = std::max<int64_t>(1, std::min(g, L.cap[q]));
        L.first[q + 1] = L.first[q] + int32_t(g);
    }
}

int64_t groups_of(const Shared &L, size_t q) { return L.first[q + 1] - L.first[q]; }

// Writes the argument table (records and workgroup ranges of every shared launch).
void fill_table(const npf_batch_s *b, char *host, const npf_tensor *A, const void *const *U,
                const void *const *V, const void *const *lam, char *ws)
{
    for (const Shared &L : b->shared) {
        Bf3Args *rec = reinterpret_cast<Bf3Args *>(host + L.args_off);
        for (size_t q = 0; q < L.sys.size(); ++q) {
            const int s = L.sys[q];
            const npf_plan_s *p = b->sys[s].plan;
            char *w = ws + b->table_bytes + b->sys[s].off;
            if (L.kind == 0) {
                const ChainArgs ca{p, L.M, 0, p->n, &A[s * (NPF_MAX_ORDER - 1) + L.M - 2],
                                   static_cast<const double *>(U[s]),
                                   static_cast<const double *>(V[s]), w, nullptr};
                rec[q] = stage_args(ca, L.i);
            } else {
                rec[q] = fused_args(p, L.M, 0, p->n, static_cast<const double *>(lam[s]), w);
            }
        }
        std::memcpy(host + L.first_off, L.first.data(), L.first.size() * sizeof(int32_t));
    }
}

int check_hip(hipError_t e, const char *where)
{
    if (e == hipSuccess) return NPF_OK;
    return fail(NPF_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

hipError_t launch_shared(const Shared &L, char *ws, hipStream_t s)
{
    MultiLaunch m{ws + L.args_off, reinterpret_cast<const int32_t *>(ws + L.first_off),
                  int(L.sys.size()), L.first.back(), L.gy, s};
    if (L.kind == 0)
        return L.npad <= 64 ? launch_stage_bf3_multi(L.npad, L.M - L.i, m)
                            : launch_stage_bf3_tr_multi(L.npad, L.M - L.i, m);
    return L.npad <= 64 ? launch_fused_bf3_multi(L.npad, L.M, m)
                        : launch_fused_bf3_tr_multi(L.npad, L.M, m);
}

// The launch sequence after the table upload.  `ev` (nullable) receives an event pair per
// shared launch for the autotuner.
int run_waves(npf_batch_s *b, const npf_tensor *A, const void *const *U, const void *const *V,
              const void *const *lam, char *ws, void *const *P_out, void *const *npf_out,
              hipStream_t st, std::vector<hipEvent_t> *ev)
{
    int rc = NPF_OK;
    for (size_t w = 0; w < b->waves.size() && rc == NPF_OK; ++w) {
        const std::vector<int> &ws_sys = b->waves[w];
        auto region = [&](int s) { return ws + b->table_bytes + b->sys[s].off; };
        for (int s : ws_sys) {
            const npf_plan_s *p = b->sys[s].plan;
            rc = check_hip(launch_prepare(p, static_cast<const double *>(U[s]),
                                          static_cast<const double *>(V[s]), nullptr, region(s), st),
                           "operand staging");
            if (rc) return rc;
        }
        for (int M = 2; M <= b->Nmax; ++M) {
            for (int s : ws_sys) {
                const npf_plan_s *p = b->sys[s].plan;
                if (p->N < M) continue;
                const npf_tensor *At = &A[s * (NPF_MAX_ORDER - 1) + M - 2];
                if (planned_tucker(p, M)) {
                    rc = check_hip(launch_tucker_rows(p, M, At, static_cast<const double *>(V[s]),
                                                      region(s), st),
                                   "per-row lower-index contraction");
                    if (!rc)
                        rc = check_hip(launch_tucker_psi(p, M, 0, p->n,
                                                         static_cast<const double *>(U[s]),
                                                         region(s), st),
                                       "upper-index contraction of the per-row tables");
                    if (rc) return rc;
                    continue;
                }
                const ChainArgs ca{p, M, 0, p->n, At, static_cast<const double *>(U[s]),
                                   static_cast<const double *>(V[s]), region(s), st};
                if ((rc = check_hip(launch_psi_a(ca), "upper-index contraction"))) return rc;
            }
            for (int pass = 0; pass < M; ++pass) {          // stages 1..M-1, then fused
                for (size_t li = 0; li < b->shared.size(); ++li) {
                    const Shared &L = b->shared[li];
                    if (L.wave != int(w) || L.M != M) continue;
                    if (pass < M - 1 ? (L.kind != 0 || L.i != pass + 1) : L.kind != 1) continue;
                    if (ev) (void)hipEventRecord((*ev)[2 * li], st);
                    if ((rc = check_hip(launch_shared(L, ws, st), "shared launch"))) return rc;
                    if (ev) (void)hipEventRecord((*ev)[2 * li + 1], st);
                }
            }
            for (size_t li = 0; li < b->shared.size(); ++li) {
                const Shared &L = b->shared[li];
                if (L.wave != int(w) || L.M != M || L.kind != 1) continue;
                for (size_t q = 0; q < L.sys.size(); ++q) {
                    const int s = L.sys[q];
                    const npf_plan_s *p = b->sys[s].plan;
                    char *r = region(s);
                    const int64_t nn = p->n * p->n;
                    double *PM = (P_out && P_out[s])
                                     ? static_cast<double *>(P_out[s]) + 2 * (M - 2) * nn
                                     : reinterpret_cast<double *>(r + p->lay.pm);
                    const int64_t slots = groups_of(L, q) *
                                          (L.npad <= 64 ? 1 : fused_bf3_tr_slices(p, p->Jpad));
                    const NpfOut fin{static_cast<const double *>(U[s]),
                                     static_cast<const double *>(V[s]),
                                     npf_out ? static_cast<double *>(npf_out[s]) : nullptr};
                    rc = check_hip(launch_reduce_parts_n(p, slots, 0, p->n, PM,
                                                         reinterpret_cast<double *>(r + p->lay.psum),
                                                         M == 2, r, st,
                                                         (M == p->N && fin.npf) ? &fin : nullptr),
                                   "partial sums");
                    if (rc) return rc;
                }
            }
        }

    }
    return rc;
}

// Eager run: upload the table from the batch's pinned staging, then the launches.
int run_eager(npf_batch_s *b, const npf_tensor *A, const void *const *U, const void *const *V,
              const void *const *lam, char *ws, void *const *P_out, void *const *npf_out,
              hipStream_t st, std::vector<hipEvent_t> *ev)
{
    if (!b->table) {           // pinned staging, made on the first eager run
        if (hipHostMalloc(&b->table, size_t(b->table_bytes), hipHostMallocDefault) != hipSuccess) {
            b->table = nullptr;
            return fail(NPF_E_DEVICE, "pinned argument staging");
        }
        if (hipEventCreateWithFlags(&b->table_done, hipEventDisableTiming) != hipSuccess) {
            b->table_done = nullptr;
            return fail(NPF_E_DEVICE, "argument staging event");
        }
    }
    if (b->table_pending) {
        if (hipEventSynchronize(b->table_done) != hipSuccess)
            return fail(NPF_E_DEVICE, "waiting for the previous argument upload");
        b->table_pending = false;
    }
    fill_table(b, static_cast<char *>(b->table), A, U, V, lam, ws);
    int rc = check_hip(hipMemcpyAsync(ws, b->table, size_t(b->table_bytes), hipMemcpyHostToDevice, st),
                       "argument upload");
    if (rc) return rc;
    if (hipEventRecord(b->table_done, st) == hipSuccess) b->table_pending = true;
    return run_waves(b, A, U, V, lam, ws, P_out, npf_out, st, ev);
}

int check_args(const npf_batch_s *b, const npf_tensor *A, const void *const *U,
               const void *const *V, const void *const *lam, void *ws, int64_t ws_bytes,
               void *const *npf_out)
{
    if (!A || !U || !V || !lam || !ws) return fail(NPF_E_INVALID, "null argument");
    if (ws_bytes < b->ws_bytes) return fail(NPF_E_INVALID, "workspace smaller than planned");
    for (size_t s = 0; s < b->sys.size(); ++s) {
        const npf_plan_s *p = b->sys[s].plan;
        if (!U[s] || !V[s] || !lam[s]) return fail(NPF_E_INVALID, "null per-system pointer");
        for (int M = 2; M <= p->N; ++M) {
            const npf_tensor *At = &A[s * (NPF_MAX_ORDER - 1) + M - 2];
            const int rc = check_tensor(p, At, M);
            if (rc) return rc;
            if (planned_tucker(p, M) && At->kind != NPF_SRC_SPARSE)
                return fail(NPF_E_INVALID, "a system with a support bound needs sparse tensors");
        }
    }
    (void)npf_out;
    return NPF_OK;
}

}  // namespace

npf_batch_s::~npf_batch_s()
{
    free_graphs(this);
    for (auto &s : sys) npf_plan_destroy(s.plan);
    // The eager staging table is read by a copy that may still be queued.
    if (table_pending && table_done) (void)hipEventSynchronize(table_done);
    if (table) (void)hipHostFree(table);
    if (table_done) (void)hipEventDestroy(table_done);
}

extern "C" int npf_batch_create(const npf_problem *problems, int64_t count, int64_t hbm_budget_bytes,
                                npf_batch_t *batch_out)
{
    if (!problems || !batch_out || count < 1) return fail(NPF_E_INVALID, "null argument or empty batch");
    if (hbm_budget_bytes < 0) return fail(NPF_E_INVALID, "negative budget");
    *batch_out = nullptr;
    npf_batch_s *b = new (std::nothrow) npf_batch_s();
    if (!b) return fail(NPF_E_INVALID, "out of host memory");
    for (int64_t s = 0; s < count; ++s) {
        npf_problem q = problems[s];
        if (q.precision != NPF_BF16X3) {
            delete b;
            return fail(NPF_E_UNSUPPORTED, "batched systems run the split-BF16 kernels only");
        }
        if (q.order_max > 4 || q.n > 256) {
            delete b;
            return fail(NPF_E_UNSUPPORTED, "batched systems need N <= 4 and n <= 256");
        }
        if (q.n_modes != 0 || q.conj_of || q.a_convention != NPF_A_DERIVATIVE) {
            delete b;
            return fail(NPF_E_UNSUPPORTED, "batched systems run all modes of derivative tensors");
        }
        q.block_modes = 0;
        q.hbm_budget_bytes = 0;
        q.flags |= NPF_FLAG_SERIAL_ORDERS;      // the batch runs each system's orders in turn
        npf_plan_t p = nullptr;
        const int rc = npf_plan_create(&q, &p);
        if (rc) {
            delete b;
            return rc;
        }
        b->sys.push_back({p, 0, 0});
        b->Nmax = std::max(b->Nmax, p->N);
        for (int M = 2; M <= p->N; ++M) b->entries += p->n * p->U[M];
    }
    // Waves: systems in order, a new wave when the next one would exceed the budget.
    int64_t used = 0;
    b->waves.emplace_back();
    for (size_t s = 0; s < b->sys.size(); ++s) {
        const int64_t need = round_up(b->sys[s].plan->lay.total, 256);
        if (hbm_budget_bytes > 0 && need > hbm_budget_bytes) {
            delete b;
            return fail(NPF_E_BUDGET, "one system alone exceeds the workspace budget");
        }
        if (hbm_budget_bytes > 0 && used + need > hbm_budget_bytes && !b->waves.back().empty()) {
            b->waves.emplace_back();
            used = 0;
        }
        b->sys[s].wave = int(b->waves.size()) - 1;
        b->sys[s].off = used;
        used += need;
        b->waves.back().push_back(int(s));
        b->wave_bytes = std::max(b->wave_bytes, used);
    }
    // Shared launches: per wave, padded size, order, and stage (or the fused last stage).
    for (size_t w = 0; w < b->waves.size(); ++w) {
        std::vector<int64_t> pads;
        for (int s : b->waves[w]) pads.push_back(b->sys[s].plan->npad);
        std::sort(pads.begin(), pads.end());
        pads.erase(std::unique(pads.begin(), pads.end()), pads.end());
        for (int64_t npad : pads)
            for (int M = 2; M <= b->Nmax; ++M)
                for (int i = 1; i <= M; ++i) {
                    Shared L;
                    L.wave = int(w);
                    L.kind = (i == M) ? 1 : 0;
                    L.npad = int(npad);
                    L.M = M;
                    L.i = i;
                    L.target = L.kind ? 512 : 1024;
                    for (int s : b->waves[w]) {
                        const npf_plan_s *p = b->sys[s].plan;
                        if (p->npad != npad || p->N < M) continue;
                        if (L.kind == 0 && planned_tucker(p, M)) continue;
                        L.sys.push_back(s);
                        L.gy = std::max<int>(L.gy, int((p->Jpad + 63) / 64));
                        const double Jn = double(p->Jpad) * double(p->n);
                        const double Jf = double(p->n) * double(p->n);
                        if (L.kind == 0) {
                            // The t-range stage takes two items per workgroup iteration.
                            const int64_t items = p->U[i - 1] * p->U[M - i];
                            L.cap.push_back(std::max<int64_t>(1, npad > 64 ? (items + 1) / 2 : items));
                            L.work.push_back(Jn * double(p->U[i]) * double(p->U[M - i]));
                            L.flops += 8.0 * Jf * double(p->U[i]) * double(p->U[M - i]);
                        } else {
                            L.cap.push_back(std::max<int64_t>(1, fused_default_groups(p, M)));
                            L.work.push_back(2.0 * Jn * double(p->U[M]));
                            L.flops += 16.0 * Jf * double(p->U[M]);
                        }
                    }
                    if (!L.sys.empty()) {
                        share_out(L);
                        b->shared.push_back(std::move(L));
                    }
                }
    }
    int64_t off = 0;
    for (Shared &L : b->shared) {
        L.args_off = off;
        off = round_up(off + int64_t(L.sys.size() * sizeof(Bf3Args)), 256);
        L.first_off = off;
        off = round_up(off + int64_t(L.first.size() * sizeof(int32_t)), 256);
    }
    b->table_bytes = std::max<int64_t>(off, 256);
    b->ws_bytes = b->table_bytes + b->wave_bytes;
    // Launches per run (about): per system prepare and per order its upper-index
    // contraction (two for sparse sources) and one partial-sum launch; plus the shared.
    int64_t per = 0;
    for (const Sys &s : b->sys) per += 1 + 3 * (s.plan->N - 1);
    b->launches = per + int64_t(b->shared.size()) + 1;
    *batch_out = b;
    return NPF_OK;
}

extern "C" int npf_batch_info(npf_batch_t b, npf_batch_report *r)
{
    if (!b || !r) return fail(NPF_E_INVALID, "null argument");
    r->systems = int64_t(b->sys.size());
    r->waves = int64_t(b->waves.size());
    r->workspace_bytes = b->ws_bytes;
    r->modal_entries = b->entries;
    r->launches = b->launches;
    r->shared_launches = int64_t(b->shared.size());
    return NPF_OK;
}

extern "C" void npf_batch_destroy(npf_batch_t b) { delete b; }

extern "C" int npf_batch_run(npf_batch_t b, const npf_tensor *A, const void *const *U,
                             const void *const *V, const void *const *lambda, void *ws,
                             int64_t ws_bytes, void *const *P_out, void *const *npf_out, void *stream)
{
    if (!b) return fail(NPF_E_INVALID, "null batch");
    int rc = check_args(b, A, U, V, lambda, ws, ws_bytes, npf_out);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    std::lock_guard<std::mutex> lock(b->mu);
    bool graph = st != nullptr;
    if (graph) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) graph = false;
    }
    if (!graph) return run_eager(b, A, U, V, lambda, w, P_out, npf_out, st, nullptr);

    const size_t S = b->sys.size();
    std::vector<uintptr_t> key;
    key.reserve(S * (5 + 3 * sizeof(npf_tensor) / sizeof(uintptr_t)) + 3);
    key.push_back(reinterpret_cast<uintptr_t>(ws));
    key.push_back(uintptr_t(ws_bytes));
    key.push_back(reinterpret_cast<uintptr_t>(st));
    for (size_t s = 0; s < S; ++s) {
        key.push_back(reinterpret_cast<uintptr_t>(U[s]));
        key.push_back(reinterpret_cast<uintptr_t>(V[s]));
        key.push_back(reinterpret_cast<uintptr_t>(lambda[s]));
        key.push_back(reinterpret_cast<uintptr_t>(P_out ? P_out[s] : nullptr));
        key.push_back(reinterpret_cast<uintptr_t>(npf_out ? npf_out[s] : nullptr));
        for (int M = 2; M <= b->sys[s].plan->N; ++M) {
            const npf_tensor &t = A[s * (NPF_MAX_ORDER - 1) + M - 2];
            uintptr_t words[sizeof(npf_tensor) / sizeof(uintptr_t) + 1] = {0};
            std::memcpy(words, &t, sizeof(npf_tensor));
            key.insert(key.end(), std::begin(words), std::end(words));
        }
    }
    for (auto &g : b->graphs)
        if (g.key == key) {
            g.used = ++b->clock;
            return launch_graph(g, st);
        }
    if (b->graphs.size() >= kMaxBatchGraphs) return run_eager(b, A, U, V, lambda, w, P_out, npf_out, st, nullptr);
    GraphEntry e;
    e.key = std::move(key);
    if (hipEventCreateWithFlags(&e.done, hipEventDisableTiming) != hipSuccess)
        return run_eager(b, A, U, V, lambda, w, P_out, npf_out, st, nullptr);
    if (hipHostMalloc(&e.table, size_t(b->table_bytes), hipHostMallocDefault) != hipSuccess) {
        (void)hipEventDestroy(e.done);
        return run_eager(b, A, U, V, lambda, w, P_out, npf_out, st, nullptr);
    }
    fill_table(b, static_cast<char *>(e.table), A, U, V, lambda, w);
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipHostFree(e.table);
        (void)hipEventDestroy(e.done);
        return run_eager(b, A, U, V, lambda, w, P_out, npf_out, st, nullptr);
    }
    rc = check_hip(hipMemcpyAsync(w, e.table, size_t(b->table_bytes), hipMemcpyHostToDevice, st),
                   "argument upload");
    if (!rc) rc = run_waves(b, A, U, V, lambda, w, P_out, npf_out, st, nullptr);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(st, &g);
    if (rc || ec != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipHostFree(e.table);
        (void)hipEventDestroy(e.done);
        return rc ? rc : check_hip(ec != hipSuccess ? ec : hipErrorUnknown, "graph capture");
    }
    const hipError_t ei = hipGraphInstantiate(&e.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
        (void)hipHostFree(e.table);
        (void)hipEventDestroy(e.done);
        return check_hip(ei, "graph instantiate");
    }
    e.used = ++b->clock;
    b->graphs.push_back(e);
    return launch_graph(b->graphs.back(), st);
}

extern "C" int npf_batch_tune(npf_batch_t b, const npf_tensor *A, const void *const *U,
                              const void *const *V, const void *const *lambda, void *ws,
                              int64_t ws_bytes, void *const *P_out, void *const *npf_out,
                              void *stream, int64_t *chosen)
{
    if (!b) return fail(NPF_E_INVALID, "null batch");
    int rc = check_args(b, A, U, V, lambda, ws, ws_bytes, npf_out);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lock(b->mu);
    const size_t nl = b->shared.size();
    std::vector<hipEvent_t> ev(2 * nl, nullptr);
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            for (auto &x : ev) if (x) (void)hipEventDestroy(x);
            return fail(NPF_E_DEVICE, "event creation");
        }
    std::vector<float> best(nl, 1e30f);
    std::vector<int64_t> best_t(nl, 0);
    for (int64_t t : kTargets) {
        for (Shared &L : b->shared) {
            L.target = t;
            share_out(L);
        }
        rc = run_eager(b, A, U, V, lambda, static_cast<char *>(ws), P_out, npf_out, st, &ev);
        if (!rc) rc = check_hip(hipStreamSynchronize(st), "tuning run");
        if (rc) break;
        for (size_t li = 0; li < nl; ++li) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, ev[2 * li], ev[2 * li + 1]) == hipSuccess && ms < best[li]) {
                best[li] = ms;
                best_t[li] = t;
            }
        }
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    for (size_t li = 0; li < nl; ++li) {
        Shared &L = b->shared[li];
        if (best_t[li]) L.target = best_t[li];
        share_out(L);
        if (chosen) chosen[li] = L.target;
    }
    free_graphs(b);
    return rc;
}

extern "C" int npf_batch_launches(npf_batch_t b, npf_batch_launch *out, int64_t cap, int64_t *count)
{
    if (!b || !count) return fail(NPF_E_INVALID, "null argument");
    *count = int64_t(b->shared.size());
    for (int64_t li = 0; out && li < cap && li < *count; ++li) {
        const Shared &L = b->shared[size_t(li)];
        out[li] = npf_batch_launch{L.wave, L.kind, L.npad, L.M, L.kind ? 0 : L.i,
                                   int32_t(L.sys.size()), int64_t(L.first.back()), L.flops,
                                   double(L.ms)};
    }
    return NPF_OK;
}

extern "C" int npf_batch_time(npf_batch_t b, const npf_tensor *A, const void *const *U,
                              const void *const *V, const void *const *lambda, void *ws,
                              int64_t ws_bytes, void *const *P_out, void *const *npf_out,
                              void *stream)
{
    if (!b) return fail(NPF_E_INVALID, "null batch");
    int rc = check_args(b, A, U, V, lambda, ws, ws_bytes, npf_out);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lock(b->mu);
    const size_t nl = b->shared.size();
    std::vector<hipEvent_t> ev(2 * nl, nullptr);
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            for (auto &x : ev) if (x) (void)hipEventDestroy(x);
            return fail(NPF_E_DEVICE, "event creation");
        }
    rc = run_eager(b, A, U, V, lambda, static_cast<char *>(ws), P_out, npf_out, st, &ev);
    if (!rc) rc = check_hip(hipStreamSynchronize(st), "timed run");
    for (size_t li = 0; li < nl && !rc; ++li) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, ev[2 * li], ev[2 * li + 1]) == hipSuccess) b->shared[li].ms = ms;
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    return rc;
}
