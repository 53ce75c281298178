// apply.hip -- stencil application and RK4 time stepping on gfx950.
//
// Operator (Sec. 2 eq. general_do of King, Lind & Nasar):
//   L^d_i(u) = sum_{j in row i} w^d_ij (u_j - u_i).
// The gather-multiply-reduce is HBM-bound: G lanes share a CSR row, the
// index and weight streams of a row are read once, contiguously, U loads per
// lane in flight before the gathers, and the partial sums are reduced across
// the G lanes with shuffles.  Several operators on the same neighbour
// structure share the index stream.
//
// Time stepping: classical RK4 (Sec. 5.1) on du/dt = L_lin(u) - gamma B(B(u)),
// with optional Dirichlet nodes whose stage derivatives are zero.
// With B present each stage is two passes: A computes L_lin(u_s) and B(u_s)
// with one read of the index stream; B applies B to that result, forms the
// stage derivative and the stage update.  Without B one pass per stage.
#include "labfm_internal.hpp"
#include "stencil_rows.hpp"

#include <cstring>

namespace labfm {

namespace {

using namespace rows;

constexpr int AOPS = 5;

template <typename T, int NOPS>
__global__ __launch_bounds__(256) void k_apply(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                               int64_t n, int64_t nnz, const T* __restrict__ w,
                                               const T* __restrict__ u, T* __restrict__ out) {
    constexpr int G = Shape<T>::G, U = Shape<T>::U;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t row = gid / G;
    const int sub = (int)(gid % G);
    if (row >= n) return;  // whole groups exit together
    WPtrs<T, NOPS> wp;
#pragma unroll
    for (int d = 0; d < NOPS; ++d) wp.p[d] = w + (int64_t)d * nnz;
    T acc[NOPS];
#pragma unroll
    for (int d = 0; d < NOPS; ++d) acc[d] = T(0);
    row_sums<T, G, U, NOPS>(col, rp[row], rp[row + 1], sub, wp, u, u[row], acc);
#pragma unroll
    for (int d = 0; d < NOPS; ++d) {
        const T v = group_sum<T, G>(acc[d]);
        if (sub == 0) out[(int64_t)d * n + row] = v;
    }
}

template <typename T>
__global__ void k_combine(const double* __restrict__ w, int nsets, double c0, double c1, double c2, double c3,
                          double c4, int64_t nnz, double* out64, float* out32) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nnz) return;
    const double c[5] = {c0, c1, c2, c3, c4};
    double acc = 0.0;
    for (int k = 0; k < nsets; ++k) acc += c[k] * w[(int64_t)k * nnz + s];
    if (out64) out64[s] = acc;
    if (out32) out32[s] = (float)acc;
}

// single pass: k = L_lin(us_in), then the stage update
template <typename T>
__global__ __launch_bounds__(256) void k_step_single(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                     int64_t n, const T* __restrict__ wl, const T* us_in, T dt,
                                                     int stage, const int8_t* __restrict__ fixed, T* u, T* acc,
                                                     T* us_out) {
    constexpr int G = Shape<T>::G, U = Shape<T>::U;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t row = gid / G;
    const int sub = (int)(gid % G);
    if (row >= n) return;
    const Rk4Node<T> node = rk4_load<T>(stage, row, fixed, u, acc);
    WPtrs<T, 1> wp{{wl}};
    T a[1] = {T(0)};
    row_sums<T, G, U, 1>(col, rp[row], rp[row + 1], sub, wp, us_in, us_in[row], a);
    const T k = group_sum<T, G>(a[0]);
    if (sub == 0) rk4_store<T>(stage, k, dt, row, node, u, acc, us_out);
}

// pass A: ra = L_lin(us_in), b1 = B(us_in), one read of the index stream
template <typename T>
__global__ __launch_bounds__(256) void k_step_a(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                int64_t n, const T* __restrict__ wl, const T* __restrict__ wb,
                                                const T* __restrict__ us_in, T* __restrict__ ra, T* __restrict__ b1) {
    constexpr int G = Shape<T>::G, U = Shape<T>::U;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t row = gid / G;
    const int sub = (int)(gid % G);
    if (row >= n) return;
    WPtrs<T, 2> wp{{wl, wb}};
    T a[2] = {T(0), T(0)};
    row_sums<T, G, U, 2>(col, rp[row], rp[row + 1], sub, wp, us_in, us_in[row], a);
    const T la = group_sum<T, G>(a[0]);
    const T lb = group_sum<T, G>(a[1]);
    if (sub == 0) {
        ra[row] = la;
        b1[row] = lb;
    }
}

// pass B: k = ra - gamma B(b1), then the stage update
template <typename T>
__global__ __launch_bounds__(256) void k_step_b(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                int64_t n, const T* __restrict__ wb, const T* __restrict__ b1,
                                                const T* __restrict__ ra, T gamma, T dt, int stage,
                                                const int8_t* __restrict__ fixed, T* u, T* acc, T* us_out) {
    constexpr int G = Shape<T>::G, U = Shape<T>::U;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t row = gid / G;
    const int sub = (int)(gid % G);
    if (row >= n) return;
    const Rk4Node<T> node = rk4_load<T>(stage, row, fixed, u, acc);
    const T rai = ra[row];
    WPtrs<T, 1> wp{{wb}};
    T c[1] = {T(0)};
    row_sums<T, G, U, 1>(col, rp[row], rp[row + 1], sub, wp, b1, b1[row], c);
    const T bb = group_sum<T, G>(c[0]);
    if (sub == 0) rk4_store<T>(stage, rai - gamma * bb, dt, row, node, u, acc, us_out);
}

template <typename T>
labfm_err enqueue_step(const labfm_step_plan* p, T* u, T* scratch, hipStream_t st) {
    const int64_t n = p->n;
    T* usA = scratch;
    T* usB = scratch + n;
    T* acc = scratch + 2 * n;
    T* ra = scratch + 3 * n;
    T* b1 = scratch + 4 * n;
    const T* in[4] = {u, usA, usB, usA};
    T* outs[4] = {usA, usB, usA, u};
    const T dt = (T)p->dt;
    const T gamma = (T)p->gamma;
    const unsigned nb = blocks_for<T>(n);
    for (int stage = 0; stage < 4; ++stage) {
        if (p->w_bh) {
            k_step_a<T><<<nb, 256, 0, st>>>(p->row_ptr, p->col, n, (const T*)p->w_lin, (const T*)p->w_bh, in[stage],
                                            ra, b1);
            k_step_b<T><<<nb, 256, 0, st>>>(p->row_ptr, p->col, n, (const T*)p->w_bh, b1, ra, gamma, dt, stage,
                                            p->fixed, u, acc, outs[stage]);
        } else {
            k_step_single<T><<<nb, 256, 0, st>>>(p->row_ptr, p->col, n, (const T*)p->w_lin, in[stage], dt, stage,
                                                 p->fixed, u, acc, outs[stage]);
        }
    }
    LABFM_HIP_CHECK(hipGetLastError());
    return LABFM_OK;
}

template <typename T>
void launch_apply(const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t nnz, int nops, const T* w,
                  const T* u, T* out, hipStream_t st) {
    const unsigned nb = blocks_for<T>(n);
    switch (nops) {
        case 1: k_apply<T, 1><<<nb, 256, 0, st>>>(row_ptr, col, n, nnz, w, u, out); break;
        case 2: k_apply<T, 2><<<nb, 256, 0, st>>>(row_ptr, col, n, nnz, w, u, out); break;
        case 3: k_apply<T, 3><<<nb, 256, 0, st>>>(row_ptr, col, n, nnz, w, u, out); break;
        case 4: k_apply<T, 4><<<nb, 256, 0, st>>>(row_ptr, col, n, nnz, w, u, out); break;
        default: k_apply<T, AOPS><<<nb, 256, 0, st>>>(row_ptr, col, n, nnz, w, u, out); break;
    }
}

}  // namespace

labfm_err apply_launch(Context* c, const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t nnz, int nops,
                       const void* w, int dtype, const void* u, void* out, hipStream_t st) {
    if (n == 0) return LABFM_OK;
    KernelTimer timer(c, dtype == 0 ? "apply_f32" : "apply_f64", st);
    if (dtype == 0)
        launch_apply<float>(row_ptr, col, n, nnz, nops, (const float*)w, (const float*)u, (float*)out, st);
    else
        launch_apply<double>(row_ptr, col, n, nnz, nops, (const double*)w, (const double*)u, (double*)out, st);
    LABFM_HIP_CHECK(hipGetLastError());
    return LABFM_OK;
}

labfm_err combine_launch(const double* w64, int nsets, const double* coef, int64_t nnz, double* out64,
                         float* out32, hipStream_t st) {
    if (nnz == 0) return LABFM_OK;
    double c[5] = {0, 0, 0, 0, 0};
    for (int k = 0; k < nsets; ++k) c[k] = coef[k];
    k_combine<double><<<(unsigned)((nnz + 255) / 256), 256, 0, st>>>(w64, nsets, c[0], c[1], c[2], c[3], c[4], nnz,
                                                                     out64, out32);
    LABFM_HIP_CHECK(hipGetLastError());
    return LABFM_OK;
}

labfm_err step_launch(Context* c, const labfm_step_plan* p, void* u, void* scratch, int nsteps, int use_graph,
                      hipStream_t st) {
    if (p->n == 0 || nsteps <= 0) return LABFM_OK;
    if (!use_graph) {
        KernelTimer timer(c, "step_direct", st);
        for (int s = 0; s < nsteps; ++s) {
            labfm_err e = p->dtype == 0 ? enqueue_step<float>(p, (float*)u, (float*)scratch, st)
                                        : enqueue_step<double>(p, (double*)u, (double*)scratch, st);
            if (e != LABFM_OK) return e;
        }
        return LABFM_OK;
    }
    // capture one step on a private stream once per (plan, buffers, stream);
    // replay the graph nsteps times on `st`
    const labfm_step_plan& k = c->step_key;  // field by field: the struct has padding
    const bool same = c->step_exec && c->step_stream == st && c->step_u == u && c->step_scratch == scratch &&
                      k.row_ptr == p->row_ptr && k.col == p->col && k.n == p->n && k.nnz == p->nnz &&
                      k.dtype == p->dtype && k.w_lin == p->w_lin && k.w_bh == p->w_bh && k.gamma == p->gamma &&
                      k.dt == p->dt && k.fixed == p->fixed;
    if (!same) {
        if (c->step_exec) LABFM_HIP_CHECK(hipStreamSynchronize(c->step_stream));
        release_step_graph(c);
        hipStream_t cap;
        LABFM_HIP_CHECK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            hipStreamDestroy(cap);
            set_error("labfm_step: hipStreamBeginCapture failed");
            return LABFM_EHIP;
        }
        labfm_err e = p->dtype == 0 ? enqueue_step<float>(p, (float*)u, (float*)scratch, cap)
                                    : enqueue_step<double>(p, (double*)u, (double*)scratch, cap);
        hipError_t he = hipStreamEndCapture(cap, &graph);
        hipGraphExec_t exec = nullptr;
        if (e == LABFM_OK && he == hipSuccess) he = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (graph) hipGraphDestroy(graph);
        hipStreamDestroy(cap);
        if (e != LABFM_OK) return e;
        if (he != hipSuccess) {
            set_error(std::string("labfm_step: graph capture: ") + hipGetErrorString(he));
            return LABFM_EHIP;
        }
        c->step_exec = exec;
        c->step_stream = st;
        c->step_u = u;
        c->step_scratch = scratch;
        c->step_key = *p;
    }
    KernelTimer timer(c, "step_graph", st);
    for (int s = 0; s < nsteps; ++s) LABFM_HIP_CHECK(hipGraphLaunch(c->step_exec, st));
    return LABFM_OK;
}

void release_step_graph(Context* c) {
    if (c->step_exec) hipGraphExecDestroy(c->step_exec);
    c->step_exec = nullptr;
    c->step_stream = nullptr;
    c->step_u = nullptr;
    c->step_scratch = nullptr;
}

}  // namespace labfm
