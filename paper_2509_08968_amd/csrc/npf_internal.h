// Internal declarations shared by the planner, the kernels and the C ABI entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "npf.h"

struct npf_plan_s;

namespace npf {

// Per-thread error message for npf_last_error().
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

// Checks a derivative-tensor descriptor of order M against a plan (NPF_OK or an error code
// with the message set).
int check_tensor(const npf_plan_s *p, const npf_tensor *A, int M);

// binom(a, b) on the host (exact; 0 outside 0 <= b <= a).
int64_t binom(int64_t a, int64_t b);

// Tables of sorted tuples of length 1..maxlen (packed 9 bits per entry), in colex order:
// the tuple of rank r and length m is entry off[m] + r.
struct TupleTables {
    int64_t count[NPF_MAX_ORDER + 1] = {0};
    int64_t off[NPF_MAX_ORDER + 1] = {0};
    int64_t total = 0;
    int maxlen = 0;
};

// Highest order the FP32 and split-BF16 paths serve (they meet their 1e-6 bound there).
constexpr int kMixedMaxOrder = 4;

// Largest per-row support of the lower-indices-first route for sparse tensors.
constexpr int kTuckerMaxSupport = 8;

// Workspace of that route (offsets in bytes; all zero when the plan has no support bound).
struct TuckerLayout {
    int64_t over = 0, S = 0, cnt = 0, inv = 0, invcnt = 0, D = 0, Y = 0, W = 0;
};

// Workspace layout of a plan.  All offsets are in bytes from the start of `ws` and are
// multiples of 256.
struct Layout {
    int64_t buf[2] = {0, 0};     // ping-pong buffers for the chain T_0 .. T_{M-1}
    int64_t buf_bytes[2] = {0, 0};
    int64_t psum = 0;            // sum of P_M over orders: [n][n] c128
    int64_t pm = 0;              // P_M of the current order: [n][n] c128
    int64_t ttab = 0;            // tuple tables
    int64_t phi = 0;             // contraction-precision copies of Phi (padded)
    int64_t phi_bytes = 0;
    int64_t parts = 0;           // per-workgroup partial P of the fused kernel
    int64_t parts_bytes = 0;
    TuckerLayout tk;
    int64_t msel = 0;            // Psi rows [nc][n] and eigenvalues [nc] of the computed
                                 // modes (c128), when the plan selects modes
    int64_t total = 0;
};

// Largest number of output modes of one call (n <= 512).
constexpr int kMaxModes = 512;
constexpr uint16_t kNoRow = 0xFFFF;

// Output rows of the computed modes c0 .. c0 + J - 1 (passed by value to the kernels that
// write P rows or read one eigenvalue per mode): row[jj] is the output mode of computed mode
// c0 + jj, conj[jj] the output mode filled with its conjugate (kNoRow: none).
struct ModeMap {
    uint16_t row[kMaxModes];
    uint16_t conj[kMaxModes];
};

}  // namespace npf

namespace npf {
// Event pairs recorded around kernel launches when profiling is on.
struct Profiler {
    bool on = false;
    struct Rec {
        std::string name;
        hipEvent_t start, stop;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t take();
    void clear();
    ~Profiler();
};
}  // namespace npf

struct npf_plan_s {
    npf_problem prob;
    int64_t n = 0;
    int N = 0;
    int prec = NPF_FP64;
    int64_t U[NPF_MAX_ORDER + 2] = {0};  // U[m] = binom(n + m - 1, m)
    int64_t J = 0;                       // output modes per block
    int64_t Jpad = 0;                    // J rounded up to a multiple of 16
    int64_t n_blocks = 0;
    int64_t npad = 0;                    // n rounded up to a multiple of 32
    int64_t esz = 16;                    // bytes per complex element of the chain
    npf::TupleTables tt;
    npf::Layout lay;                     // the layout launches read (see OrderLayout)
    npf::Profiler prof;
    // Concurrent orders: each order's chain buffers, partials, P scratch and per-row tables
    // in workspace of its own (ord[M]); the shared parts (tuple tables, operands, psum) are
    // common.  The side streams and events of the concurrent capture belong to the library
    // (one set per device), not to the plan.
    bool concurrent = false;
    npf::Layout ord[NPF_MAX_ORDER + 1];
    // Computed modes in block order (cm) and the output mode each fills by conjugation (cj,
    // -1 for none); nc = cm.size().  `select` is true unless cm = 0..n-1 with no fills, and
    // then the Psi rows and eigenvalues of the computed modes are staged in the workspace.
    int64_t nc = 0;
    std::vector<int32_t> cm, cj;
    int64_t n_out = 0;                   // output modes (computed + filled)
    bool select = false;
    // Factor applied to every P_M (and staged C): 1, or M! for Taylor-coefficient input.
    double a_scale[NPF_MAX_ORDER + 1] = {1, 1, 1, 1, 1, 1, 1};
};

namespace npf {
// While alive, launches of order M read the order's own layout (concurrent plans).
struct OrderLayout {
    npf_plan_s *plan;
    Layout saved;
    OrderLayout(npf_plan_s *p, int M) : plan(p), saved(p->lay)
    {
        if (p->concurrent) p->lay = p->ord[M];
    }
    ~OrderLayout() { plan->lay = saved; }
};
}  // namespace npf

namespace npf {
// While alive, launches for a block of J modes use the block's own width: a last block
// narrower than the others runs with Jpad = J rounded up to 16 (the layout fits any).
struct BlockShape {
    npf_plan_s *plan;
    int64_t saved;
    BlockShape(npf_plan_s *p, int64_t J) : plan(p), saved(p->Jpad)
    {
        const int64_t w = (J + 15) / 16 * 16;
        if (w < p->Jpad) p->Jpad = w;
    }
    ~BlockShape() { plan->Jpad = saved; }
};
}  // namespace npf

namespace npf {
// Brackets one kernel launch with an event pair when the plan is profiling.
struct Timed {
    npf_plan_s *plan;
    std::string name;
    hipStream_t stream;
    hipEvent_t start = nullptr;
    Timed(const npf_plan_s *p, std::string n, hipStream_t s);
    ~Timed();
};
}  // namespace npf

namespace npf {

// Kernel launchers (npf_kernels.hip).  All enqueue on `stream` and return hipError_t.
struct ChainArgs {
    const npf_plan_s *plan;
    int M;                    // order
    int64_t j0, J;            // block's first mode and its number of modes
    const npf_tensor *A;
    const double *U;          // Psi, complex128 interleaved
    const double *V;          // Phi
    char *ws;
    hipStream_t stream;
};

// Lower indices first for a sparse A_M whose rows involve at most support_max states:
// per-row support lists and tables, and W (once per order); then T_{M-1} for a block.
bool tucker_route(const npf_plan_s *p, int M);              // the plan takes the route for order M
bool tucker_supported(const npf_plan_s *p, const npf_tensor *A, int M);
hipError_t launch_tucker_rows(const npf_plan_s *p, int M, const npf_tensor *A, const double *V,
                              char *ws, hipStream_t s);
hipError_t launch_tucker_support(const npf_plan_s *p, int M, const npf_tensor *A, char *ws,
                                 hipStream_t s);
hipError_t launch_tucker_w(const npf_plan_s *p, int M, const double *V, char *ws, hipStream_t s);
hipError_t launch_tucker_psi(const npf_plan_s *p, int M, int64_t j0, int64_t J, const double *U,
                             char *ws, hipStream_t s);

// G = Psi[j0:j0+J, :] A_M over sorted tuples, into buffer 0 (T_0).
hipError_t launch_psi_a(const ChainArgs &a);
// Rows [k0, k0 + rows) of a hash-generated tensor into out[(k - k0)*UM + r].
hipError_t launch_hash_fill(double *out, uint64_t seed, double scale, int M, int64_t k0,
                            int64_t rows, int64_t UM, hipStream_t s);
// Stage i (1 <= i <= M-1) of the lower-index chain: T_{i-1} -> T_i.
hipError_t launch_stage(const ChainArgs &a, int i);
// Last stage, writes C (complex128, [J][U_M], scaled by 1/M!) to C_out.
hipError_t launch_last_to_c(const ChainArgs &a, double *C_out);
// h = C / D in place on [J][U_M].
hipError_t launch_normal_form(const npf_plan_s *p, int M, int64_t j0, int64_t J,
                              const double *lam, double *C, hipStream_t s);
// P_acc[j0+jj][k] += -sum_t m(t) h[jj][t] prod zeta_k[t_i]  (deterministic per entry).
hipError_t launch_assemble(const npf_plan_s *p, int M, int64_t j0, int64_t J, const double *h,
                           const double *U, double *P_acc, hipStream_t s);
// NPF = Phi o (delta Psi + P_sum)^T.
hipError_t launch_finalize(const npf_plan_s *p, const double *U, const double *V,
                           const double *P_sum, double *npf_out, hipStream_t s);
// Operand copies for the MFMA kernels (zero padded, in the plan's precision) and the
// tuple tables.
hipError_t launch_prepare(const npf_plan_s *p, const double *U, const double *V,
                          const double *lam, char *ws, hipStream_t s,
                          const double *zadd = nullptr);
// Output rows of computed modes [c0, c0 + J).
ModeMap mode_map(const npf_plan_s *p, int64_t c0, int64_t J);
// Psi rows and eigenvalue of the computed modes: the staged copies when the plan selects
// modes, else the caller's arrays.
const double *psi_rows(const npf_plan_s *p, const double *U, const char *ws);
const double *lam_rows(const npf_plan_s *p, const double *lam, const char *ws);
// Fused last mode product + divisor + division + reduction: per-workgroup partial P.
hipError_t launch_fused_last(const npf_plan_s *p, int M, int64_t j0, int64_t J, const double *lam,
                             char *ws, hipStream_t s);
// Sum of the partials of launch_fused_last into rows [j0, j0+J) of P (fixed order), and
// psum = P (first order) or psum += P.
// The NPF output written by the last order's partial sums (Alg. 2 step 20).
struct NpfOut {
    const double *U, *V;      // Psi, Phi
    double *npf;
};
// With inpf (interaction pass, eq. (8)): writes inpf[k*n + j] = -Phi[k,j] * (the sum) for
// the block's modes (and their conjugate fills) and nothing else; fin must then carry Phi
// (fin->npf may be null).
hipError_t launch_reduce_parts(const npf_plan_s *p, int M, int64_t j0, int64_t J, double *P,
                               double *psum, bool first, char *ws, hipStream_t s,
                               const NpfOut *fin = nullptr, double *inpf = nullptr);
int64_t fused_groups(const npf_plan_s *p, int M);
// Most partial-P slots any order writes for a block of Jpad modes.
int64_t fused_max_slots(const npf_plan_s *p, int64_t Jpad);
// Split-BF16 kernels with LDS-resident operands for npad <= 64.
bool bf3_small_supported(const npf_plan_s *p);
hipError_t launch_fused_bf3(const npf_plan_s *p, int M, int64_t j0, int64_t J, const double *lam,
                            char *ws, int64_t groups, hipStream_t s);
hipError_t launch_stage_bf3(const ChainArgs &a, int i);
hipError_t launch_stage_bf3_small(const ChainArgs &a, int i);

// One launch over several systems of the same padded size: system s runs on workgroups
// [first[s], first[s+1]) of grid.x (at least one each) with the kernel arguments args[s].
struct MultiLaunch {
    const void *args;         // device: kernel argument records [nsys]
    const int32_t *first;     // device: [nsys + 1]
    int nsys;
    int64_t groups;           // first[nsys]
    int gy;                   // 64-mode groups of the largest block
    hipStream_t stream;
};
hipError_t launch_fused_bf3_multi(int npad, int M, const MultiLaunch &m);
hipError_t launch_fused_bf3_tr_multi(int npad, int M, const MultiLaunch &m);
hipError_t launch_stage_bf3_multi(int npad, int suf, const MultiLaunch &m);
hipError_t launch_stage_bf3_tr_multi(int npad, int suf, const MultiLaunch &m);
int fused_bf3_tr_kranges(int64_t npad);
int stage_bf3_tr_tiles(int64_t npad);
// Partial sums of a block's fused-kernel slots (nparts of them) into P rows and psum.
hipError_t launch_reduce_parts_n(const npf_plan_s *p, int64_t nparts, int64_t j0, int64_t J,
                                 double *P, double *psum, bool first, char *ws, hipStream_t s,
                                 const NpfOut *fin = nullptr, double scale = 1.0,
                                 double *inpf = nullptr);
int64_t fused_default_groups(const npf_plan_s *p, int M);
bool bf3_tr_fused_supported(const npf_plan_s *p);
int bf3_items_per_group(int64_t Jpad);
int64_t fused_bf3_tr_slices(const npf_plan_s *p, int64_t Jpad);
hipError_t launch_fused_bf3_tr(const npf_plan_s *p, int M, int64_t j0, int64_t J,
                               const double *lam, char *ws, int64_t groups, hipStream_t s);
bool bf3_stage_supported(const npf_plan_s *p);
// MFMA upper-index contraction for dense tensors.
bool psi_a_mfma_supported(const npf_plan_s *p);
hipError_t launch_psi_a_mfma(const ChainArgs &a);
// MFMA version of one chain stage (n <= 512).
bool stage_mfma_supported(const npf_plan_s *p);
hipError_t launch_stage_mfma(const ChainArgs &a, int i);
// The launch sequence of npf_run, eagerly (no graph, orders in sequence), on workspace ws
// of ws_bytes bytes, after npf_run's argument checks.
int run_eager_checked(npf_plan_s *plan, const npf_tensor *A, const void *U, const void *V,
                      const void *lambda, void *ws, int64_t ws_bytes, void *P_out, void *npf_out,
                      hipStream_t s);
// Fill `count` doubles with zero.
hipError_t launch_zero(double *x, int64_t count, hipStream_t s);
// dst[i] += src[i] (or dst = src when first), count doubles.
hipError_t launch_accumulate(double *dst, const double *src, int64_t count, bool first,
                             hipStream_t s);
// Copy rows [j0, j0+J) of an n x n complex matrix.
hipError_t launch_copy_rows(double *dst, const double *src, int64_t n, int64_t j0, int64_t J,
                            hipStream_t s);

}  // namespace npf
