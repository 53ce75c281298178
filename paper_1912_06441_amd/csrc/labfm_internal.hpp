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
    // cached RK4 step graph (replayed while plan, buffers and stream are unchanged)
    hipGraphExec_t step_exec = nullptr;
    hipStream_t step_stream = nullptr;
    labfm_step_plan step_key{};
    void* step_u = nullptr;
    void* step_scratch = nullptr;
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
labfm_err neighbours_fill(Context* c, const double* x, const double* y, int64_t n, const GridSpec& g,
                          const double* R, const int64_t* row_ptr, int32_t* col, hipStream_t st);

// ---- weights
struct WeightArgs {
    const double* x;
    const double* y;
    const double* R;
    const int8_t* order;
    const int64_t* row_ptr;
    const int32_t* col;
    int64_t n, nnz;
    double Lx, Ly;
    int perx, pery;
    int abf, rbf;
    double sigma;
    unsigned ops;
    int nops;
    double tol_stop, tol_pass;
    int max_iters;
    double* w64;
    float* w32;
    int8_t* status;
    float* resid;
    int8_t* iters;
    int iters_offset;  // added to iters (marks nodes recomputed on the FP64 path)
    int max_iters32;   // refinement updates allowed on the mixed path
    const float* psi0; // warm start of the mixed path: Psi0 of node i at psi0[i * psi0_ld] (or NULL)
    int psi0_order;    // order of the nodes that use psi0
    int psi0_ld;
};
labfm_err weights_fp64(Context* c, const WeightArgs& a, hipStream_t st);
labfm_err build_order_lists(Context* c, const int8_t* order, int64_t n, hipStream_t st, int32_t** list,
                            int32_t** off, int32_t** cnt);
labfm_err weights_invalid_orders(const WeightArgs& a, const int32_t* list, const int32_t* off, const int32_t* cnt,
                                 hipStream_t st);
// FP64 kernels over given per-order lists (segment K at list + off[K], cnt[K] entries)
labfm_err weights_fp64_lists(Context* c, const WeightArgs& a, const int32_t* list, const int32_t* off,
                             const int32_t* cnt, hipStream_t st);
labfm_err weights_mixed(Context* c, const WeightArgs& a, hipStream_t st);

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
labfm_err weights_mlp(Context* c, const WeightArgs& a, const labfm_mlp* net, hipStream_t st);

// ---- application and time stepping
labfm_err apply_launch(Context* c, const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t nnz, int nops,
                       const void* w, int dtype, const void* u, void* out, hipStream_t st);
labfm_err combine_launch(const double* w64, int nsets, const double* coef, int64_t nnz, double* out64,
                         float* out32, hipStream_t st);
labfm_err step_launch(Context* c, const labfm_step_plan* plan, void* u, void* scratch, int nsteps,
                      int use_graph, hipStream_t st);

}  // namespace labfm
