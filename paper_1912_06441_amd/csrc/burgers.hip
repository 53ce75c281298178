// burgers.hip -- viscous Burgers' equation (Sec. 5.3 of King, Lind & Nasar)
// on gfx950 with classical RK4 (Sec. 5.1):
//   du/dt = -(u L^x(u) + v L^y(u)) + nu L^L(u) + L^hv(u)
//   dv/dt = -(u L^x(v) + v L^y(v)) + nu L^L(v) + L^hv(v)
// with nu = 1/Re and an optional hyperviscosity operator L^hv (Sec. 4.2) whose
// coefficient is folded into its weights; Dirichlet nodes hold their values or
// follow imposed stage derivatives.  One pass per RK4 stage: each CSR
// row reads its index stream and the 3 (or 4) weight streams once and gathers
// both velocity components, so the nonlinear right-hand side and the stage
// update of both fields come out of a single HBM-bound sweep.  Every stage
// reads its state as (u, v) pairs (the step's starting fields are packed so
// first), so a single load fetches both components of a neighbour.  One step
// is captured as a HIP graph and replayed.
#include "labfm_internal.hpp"
#include "stencil_rows.hpp"

namespace labfm {

namespace {

using namespace rows;

// the step's starting fields (u, v) as pairs, the input of the first stage
template <typename T>
__global__ __launch_bounds__(256) void k_pack_pairs(int64_t n, const T* __restrict__ u, const T* __restrict__ v,
                                                    typename Vec2<T>::type* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = typename Vec2<T>::type{u[i], v[i]};
}

template <typename T, int NW>
__global__ __launch_bounds__(256) void k_burgers_stage(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                       int64_t n, WPtrs<T, NW> w,
                                                       const typename Vec2<T>::type* __restrict__ pin, T nu, T dt,
                                                       int stage, const int8_t* __restrict__ fixed,
                                                       const T* __restrict__ dfix, T* u, T* v, T* accu, T* accv,
                                                       typename Vec2<T>::type* __restrict__ pout) {
    constexpr int G = Shape<T>::G, U = Shape<T>::U;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t row = gid / G;
    const int sub = (int)(gid % G);
    if (row >= n) return;  // whole groups exit together
    const typename Vec2<T>::type pi = pin[row];
    const T ui = pi.x, vi = pi.y;
    const Rk4Node<T> nu_ = rk4_load<T>(stage, row, fixed, u, accu, dfix ? dfix + (int64_t)stage * n : nullptr);
    const Rk4Node<T> nv_ = rk4_load<T>(stage, row, fixed, v, accv, dfix ? dfix + (int64_t)(4 + stage) * n : nullptr);
    T au[NW], av[NW];
#pragma unroll
    for (int d = 0; d < NW; ++d) au[d] = av[d] = T(0);
    row_sums2p<T, G, U, NW>(col, rp[row], rp[row + 1], sub, w, pin, ui, vi, au, av);
#pragma unroll
    for (int d = 0; d < NW; ++d) {
        au[d] = group_sum<T, G>(au[d]);
        av[d] = group_sum<T, G>(av[d]);
    }
    if (sub != 0) return;
    T ku = -(ui * au[0] + vi * au[1]) + nu * au[2];
    T kv = -(ui * av[0] + vi * av[1]) + nu * av[2];
    if (NW == 4) {
        ku += au[NW - 1];
        kv += av[NW - 1];
    }
    const T su = rk4_stage<T>(stage, ku, dt, row, nu_, u, accu);
    const T sv = rk4_stage<T>(stage, kv, dt, row, nv_, v, accv);
    if (stage < 3) pout[row] = typename Vec2<T>::type{su, sv};
}

template <typename T, int NW>
void launch_stages(const labfm_burgers_plan* p, WPtrs<T, NW> w, T* u, T* v, T* scratch, hipStream_t st) {
    using T2 = typename Vec2<T>::type;
    const int64_t n = p->n;
    // scratch: two arrays of (u, v) pairs, then the RK4 accumulators of each
    // field.  PB first holds the step's starting fields, read by stage 0 only.
    T2* PA = (T2*)scratch;
    T2* PB = (T2*)(scratch + 2 * n);
    T* au = scratch + 4 * n;
    T* av = scratch + 5 * n;
    const T dt = (T)p->dt, nu = (T)p->nu;
    const T* dfix = (const T*)p->dfix;
    const unsigned nb = blocks_for<T>(n);
    const T2* in[4] = {PB, PA, PB, PA};
    T2* out[4] = {PA, PB, PA, nullptr};
    k_pack_pairs<T><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, u, v, PB);
    for (int stage = 0; stage < 4; ++stage)
        k_burgers_stage<T, NW><<<nb, 256, 0, st>>>(p->row_ptr, p->col, n, w, in[stage], nu, dt, stage, p->fixed, dfix,
                                                   u, v, au, av, out[stage]);
}

template <typename T>
labfm_err enqueue_burgers(const labfm_burgers_plan* p, T* u, T* v, T* scratch, hipStream_t st) {
    if (p->w_hv)
        launch_stages<T, 4>(p, WPtrs<T, 4>{{(const T*)p->w_x, (const T*)p->w_y, (const T*)p->w_lap, (const T*)p->w_hv}},
                            u, v, scratch, st);
    else
        launch_stages<T, 3>(p, WPtrs<T, 3>{{(const T*)p->w_x, (const T*)p->w_y, (const T*)p->w_lap}}, u, v, scratch,
                            st);
    LABFM_HIP_CHECK(hipGetLastError());
    return LABFM_OK;
}

labfm_err enqueue_any(const labfm_burgers_plan* p, void* u, void* v, void* scratch, hipStream_t st) {
    return p->dtype == 0 ? enqueue_burgers<float>(p, (float*)u, (float*)v, (float*)scratch, st)
                         : enqueue_burgers<double>(p, (double*)u, (double*)v, (double*)scratch, st);
}

bool same_plan(const labfm_burgers_plan& a, const labfm_burgers_plan& b) {
    return a.row_ptr == b.row_ptr && a.col == b.col && a.n == b.n && a.nnz == b.nnz && a.dtype == b.dtype &&
           a.w_x == b.w_x && a.w_y == b.w_y && a.w_lap == b.w_lap && a.w_hv == b.w_hv && a.nu == b.nu &&
           a.dt == b.dt && a.fixed == b.fixed && a.dfix == b.dfix;
}

}  // namespace

labfm_err burgers_launch(Context* c, const labfm_burgers_plan* p, void* u, void* v, void* scratch, int nsteps,
                         int use_graph, hipStream_t st) {
    if (p->n == 0 || nsteps <= 0) return LABFM_OK;
    if (!use_graph) {
        KernelTimer timer(c, "burgers_direct", st);
        for (int s = 0; s < nsteps; ++s) {
            labfm_err e = enqueue_any(p, u, v, scratch, st);
            if (e != LABFM_OK) return e;
        }
        return LABFM_OK;
    }
    Context::StepGraph& g = c->burgers;
    const bool same = g.exec && g.stream == st && g.u == u && g.v == v && g.scratch == scratch &&
                      same_plan(c->burgers_key, *p);
    if (!same) {
        if (g.exec) LABFM_HIP_CHECK(hipStreamSynchronize(g.stream));
        release_burgers_graph(c);
        hipStream_t cap;
        LABFM_HIP_CHECK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            hipStreamDestroy(cap);
            set_error("labfm_burgers_step: hipStreamBeginCapture failed");
            return LABFM_EHIP;
        }
        labfm_err e = enqueue_any(p, u, v, scratch, cap);
        hipError_t he = hipStreamEndCapture(cap, &graph);
        hipGraphExec_t exec = nullptr;
        if (e == LABFM_OK && he == hipSuccess) he = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (graph) hipGraphDestroy(graph);
        hipStreamDestroy(cap);
        if (e != LABFM_OK) return e;
        if (he != hipSuccess) {
            set_error(std::string("labfm_burgers_step: graph capture: ") + hipGetErrorString(he));
            return LABFM_EHIP;
        }
        g.exec = exec;
        g.stream = st;
        g.u = u;
        g.v = v;
        g.scratch = scratch;
        c->burgers_key = *p;
    }
    KernelTimer timer(c, "burgers_graph", st);
    for (int s = 0; s < nsteps; ++s) LABFM_HIP_CHECK(hipGraphLaunch(g.exec, st));
    return LABFM_OK;
}

void release_burgers_graph(Context* c) {
    Context::StepGraph& g = c->burgers;
    if (g.exec) hipGraphExecDestroy(g.exec);
    g = Context::StepGraph{};
}

}  // namespace labfm
