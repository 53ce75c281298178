// labfm_internal.hpp -- shared declarations of the HIP library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/labfm.h"

namespace labfm {

// thread-local last error message
void set_error(const std::string& msg);

#define LABFM_HIP_CHECK(expr)                                                           \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            ::labfm::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));      \
            return LABFM_EHIP;                                                          \
        }                                                                               \
    } while (0)

// Library scratch owned by a context, grown on demand.
struct Scratch {
    void* p = nullptr;
    size_t bytes = 0;
};

struct Context {
    int device = 0;
    Scratch grid_count;   // per-cell counters / starts (int32)
    Scratch grid_idx;     // node indices sorted by cell (int32)
    Scratch node_cell;    // cell of each node (int32)
    Scratch counts;       // neighbour counts (int64)
    Scratch scan_tmp;     // block sums for scans
    Scratch worklist;     // per-order work lists (int32) + counters
    Scratch mixed;        // mixed-precision retry list
    Scratch mlp_act;      // network activations (two [B][max width] FP32 buffers)
    Scratch mlp_feat;     // stencil features of one chunk of nodes
    Scratch mlp_psi;      // network output Psi0 of every node [n][outputs]
    Scratch mlp_part;     // column-sum partials of the bias gradients
    Scratch poisson;      // reduction partials and scalars of the Krylov solve
    Scratch factors;      // LU factors, scales, pivots and Psi of one chunk of FP64 node systems
    Scratch factors3;     // the same for the three-dimensional node systems (orders 1..4)
    // cached RK4 step graph (replayed while plan, buffers and stream are unchanged)
    hipGraphExec_t step_exec = nullptr;
    hipStream_t step_stream = nullptr;
    labfm_step_plan step_key{};
    void* step_u = nullptr;
    void* step_scratch = nullptr;
    // cached Burgers step graph (same replay rule)
    struct StepGraph {
        hipGraphExec_t exec = nullptr;
        hipStream_t stream = nullptr;
        void *u = nullptr, *v = nullptr, *scratch = nullptr;
    } burgers;
    labfm_burgers_plan burgers_key{};
    // cached batched-weights graph (replayed while sets, options and stream are unchanged)
    struct Batch {
        std::vector<labfm_node_set> sets;
        labfm_wopts opt{};
        hipStream_t stream = nullptr;
        unsigned fp64_orders = 0;
        Scratch d_sets, d_off, wl, rl;  // owned by the graph
        Scratch factors;                // the FP64 factor workspace its graph writes
        hipGraphExec_t exec = nullptr;
    } batch;
    // autotuned route of each order on the mixed path, per (abf, rbf, ops)
    struct Tuned {
        int abf, rbf;
        unsigned ops;
        int order;
        int route;  // 1 mixed kernels, 2 FP64 kernels
        double ms_mixed, ms_fp64;
        int64_t sample;
    };
    std::vector<Tuned> tuned;
    // kernel timing (HIP events recorded on the launch stream around each kernel)
    bool timing = false;
    struct Timed {
        std::string name;
        hipEvent_t a, b;
    };
    std::vector<Timed> timed;
};

// Records events around the kernels launched in its scope when timing is on.
struct KernelTimer {
    Context* c;
    const char* name;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    KernelTimer(Context* ctx, const char* nm, hipStream_t stream) : c(ctx), name(nm), st(stream) {
        if (!c || !c->timing) return;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
            a = b = nullptr;
            return;
        }
        (void)hipEventRecord(a, st);
    }
    ~KernelTimer() {
        if (!a) return;
        (void)hipEventRecord(b, st);
        c->timed.push_back({name, a, b});
    }
};

void release_step_graph(Context* c);
void release_burgers_graph(Context* c);
void release_batch(Context* c);

labfm_err ensure(Scratch& s, size_t bytes);

// ---- scans (int64 exclusive scan of int64 counts, writes out[n] = total)
labfm_err exclusive_scan_i64(Context* c, const int64_t* in, int64_t* out, int64_t n, hipStream_t st);
labfm_err exclusive_scan_i32(Context* c, const int32_t* in, int32_t* out, int64_t n, hipStream_t st);

// ---- neighbours
struct GridSpec {
    int ncx, ncy;
    double lox, loy, wx, wy, Lx, Ly;
    int perx, pery;
};
labfm_err neighbours_count(Context* c, const double* x, const double* y, int64_t n, const GridSpec& g,
                           double* R, const int8_t* order, int grow, int max_grow, int64_t* row_ptr,
                           hipStream_t st);
// rows of a CSR structure sorted ascending in place (entries distinct)
labfm_err sort_rows(const int64_t* row_ptr, int32_t* col, int64_t n, hipStream_t st);
// three dimensions
struct Grid3 {
    int nc[3];
    double lo[3], w[3], L[3];
    int per[3];
};
labfm_err neighbours3_count(Context* c, const double* x, const double* y, const double* z, int64_t n,
                            const Grid3& g, const double* R, int64_t* row_ptr, hipStream_t st);
labfm_err neighbours3_fill(Context* c, const double* x, const double* y, const double* z, int64_t n,
                           const Grid3& g, const double* R, const int64_t* row_ptr, int32_t* col, hipStream_t st);
labfm_err weights3(Context* c, const double* x, const double* y, const double* z, int64_t n, const Grid3& g,
                   const double* R, int k, const int64_t* row_ptr, const int32_t* col, int64_t nnz,
                   const labfm_wopts* opt, double* w64, int8_t* status, float* resid, int8_t* iters,
                   hipStream_t st);
labfm_err neighbours_fill(Context* c, const double* x, const double* y, int64_t n, const GridSpec& g,
                          const double* R, const int64_t* row_ptr, int32_t* col, hipStream_t st);

// ---- weights
// Arrays, domain and outputs of one node set.
struct NodeSet {
    const double* x;
    const double* y;
    const double* R;
    const int8_t* order;
    const int64_t* row_ptr;
    const int32_t* col;
    int64_t n, nnz;
    double Lx, Ly;
    int perx, pery;
    double* w64;
    float* w32;
    int8_t* status;
    float* resid;
    int8_t* iters;
    const float* psi0;  // warm start: Psi0 of node i at psi0[i * psi0_ld] (or NULL)
};

// A weight computation over one node set (nsets == 1: `one`) or a batch
// (nsets > 1: device table `sets`, set s owning global work indices
// [set_off[s], set_off[s+1])).  Work lists hold global indices.
struct WeightArgs {
    NodeSet one;
    const NodeSet* sets;
    const int64_t* set_off;
    int nsets;
    int64_t ntotal;
    int abf, rbf;
    double sigma;
    unsigned ops;
    int nops;
    double tol_stop, tol_pass;
    int max_iters;
    int iters_offset;  // added to iters (marks nodes recomputed on the FP64 path)
    int max_iters32;   // refinement updates allowed on the mixed path
    int psi0_order;    // order of the nodes that use NodeSet::psi0
    int psi0_ld;
};
constexpr unsigned ALL_ORDERS = 0x1FEu;  // bits 1..8
constexpr int KMAX_ORDERS = LABFM_MAX_ORDER;
void set_options(WeightArgs& a, const labfm_wopts* opt);
void init_weight_grids();
void init_mixed_grids();
labfm_err weights_batched(Context* c, int nsets, const labfm_node_set* sets, const labfm_wopts* opt, int use_graph,
                          hipStream_t st);
labfm_err autotune_query(Context* c, int abf, int rbf, unsigned ops, int order, int* route, double* ms_mixed,
                         double* ms_fp64, int64_t* sample);
// lists: *list holds the caller's buffer (>= ntotal + 3 (KMAX + 2) int32) on entry
labfm_err build_order_lists(Context* c, const WeightArgs& a, const NodeSet* host_sets, hipStream_t st,
                            int32_t** list, int32_t** off, int32_t** cnt);
labfm_err fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st);
labfm_err weights_invalid_orders(const WeightArgs& a, const int32_t* list, const int32_t* off, const int32_t* cnt,
                                 hipStream_t st);
// FP64 kernels of the orders in `mask` over given per-order lists (segment K at list + off[K], cnt[K] entries)
labfm_err weights_fp64_lists(Context* c, const WeightArgs& a, const int32_t* list, const int32_t* off,
                             const int32_t* cnt, unsigned mask, hipStream_t st);
// whole computations; host_sets: host copy of the set table (nsets entries, or &a.one)
labfm_err weights_fp64(Context* c, const WeightArgs& a, const NodeSet* host_sets, int32_t* wl, hipStream_t st);
// the same FP64 weights in two kernels per order (factor, then weights and refinement), the
// factors of each chunk of nodes passing through the workspace ws (grown by ensure() as needed:
// reserve it with fp64_split_reserve, and the grids with init_split_grids, before a graph capture)
labfm_err weights_fp64_split_lists(Context* c, const WeightArgs& a, const int32_t* list, const int32_t* off,
                                   const int32_t* cnt, unsigned mask, Scratch& ws, hipStream_t st);
labfm_err weights_fp64_split(Context* c, const WeightArgs& a, const NodeSet* host_sets, int32_t* wl, Scratch& ws,
                             hipStream_t st);
labfm_err fp64_split_reserve(Scratch& ws, int64_t ntotal);
void init_split_grids();
// mixed kernels for the orders not in fp64_orders, FP64 kernels for those and for the retry list
// (the two-kernel FP64 route through fp64_ws when given, else the single FP64 kernel, which
// allocates nothing); direct_order (1..8, needs NodeSet::psi0): that order takes the warm start's
// Psi0 without a factorisation, its nodes above tol_pass go to the retry list.
// rl: >= ntotal + KMAX + 2 int32
labfm_err weights_mixed(Context* c, const WeightArgs& a, const NodeSet* host_sets, int32_t* wl, int32_t* rl,
                        unsigned fp64_orders, hipStream_t st, int direct_order = 0, Scratch* fp64_ws = nullptr);
labfm_err weights_mixed_lists(Context* c, const WeightArgs& a, const int32_t* list, const int32_t* off,
                              const int32_t* cnt, int32_t* rl, unsigned mask, hipStream_t st, int direct_order = 0,
                              Scratch* fp64_ws = nullptr);

// ---- learned warm start
labfm_err mlp_features(Context* c, const double* x, const double* y, const double* R, const int64_t* row_ptr,
                       const int32_t* col, int64_t first, int64_t count, double Lx, double Ly, int perx, int pery,
                       int kmax, float* feat, hipStream_t st);
size_t mlp_cache_floats(const labfm_mlp* net, int64_t B);
labfm_err mlp_forward(Context* c, const labfm_mlp* net, const float* in, int64_t B, float* out, float* cache,
                      int denorm, hipStream_t st);
labfm_err mlp_backward(Context* c, const labfm_mlp* net, const float* in, const float* cache, const float* dout,
                       int64_t B, const labfm_mlp_grads* gr, hipStream_t st);
labfm_err mlp_moment_loss(Context* c, const float* y, const float* M, const float* mu, const float* sd, int order,
                          unsigned opbits, int64_t B, float* dy, double* loss, hipStream_t st);
labfm_err mlp_adam(Context* c, float* p, const float* g, float* m, float* v, void* pb, int64_t n, const labfm_adam* hp,
                   int64_t t, hipStream_t st);
labfm_err mlp_cast_bf16(const float* src, void* dst, int64_t n, hipStream_t st);
// training data of the warm start: M (FP32 [n][p][p]) and Psi (FP32 [n][nops p]) of every node, order k
labfm_err moment_systems(Context* c, const WeightArgs& a, int k, float* M, float* psi, int8_t* status,
                         hipStream_t st);
// learned warm start: refine from the network's Psi0 with the FP32 factors (direct = false), or
// take Psi0 without a factorisation and solve the nodes it leaves above tol_pass on the FP64 path
labfm_err weights_mlp(Context* c, const WeightArgs& a, int32_t* wl, int32_t* rl, const labfm_mlp* net,
                      hipStream_t st, bool direct = false);

// ---- application and time stepping
labfm_err apply_launch(Context* c, const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t nnz, int nops,
                       const void* w, int dtype, const void* u, void* out, hipStream_t st);
labfm_err combine_launch(const double* w64, int nsets, const double* coef, int64_t nnz, double* out64,
                         float* out32, hipStream_t st);
labfm_err step_launch(Context* c, const labfm_step_plan* plan, void* u, void* scratch, int nsteps,
                      int use_graph, hipStream_t st);
labfm_err burgers_launch(Context* c, const labfm_burgers_plan* plan, void* u, void* v, void* scratch, int nsteps,
                         int use_graph, hipStream_t st);
labfm_err poisson_solve(Context* c, const labfm_poisson_plan* plan, const double* F, double* phi, double* scratch,
                        int* iters, double* rel_resid, int* converged, hipStream_t st);
labfm_err neumann_rows(Context* c, const int64_t* rp, const int32_t* col, int64_t n, const double* wx,
                       const double* wy, const double* wl, const int32_t* parent, const double* nx, const double* ny,
                       int64_t* orp, int32_t* ocol, double* ow, int32_t* ocenter, int64_t* nnz_host, hipStream_t st);
labfm_err ns_step(Context* c, const labfm_ns_plan* plan, double* omega, double* psi, double* scratch, int nsteps,
                  int* solver_iters, int* all_converged, hipStream_t st);

}  // namespace labfm
