// batch.hip -- weights of many independent node sets (Sec. 3.1 per node) in
// one launch sequence: per-order work lists over every set, one persistent
// kernel per order, the FP64 fallback, all captured as one HIP graph.
//
// Route autotuning (mixed precision): the first time an order is met under
// (abf, rbf, ops), the mixed route (matrix-core assembly, FP32 LU, FP64
// refinement, FP64 retries) and the FP64 route are timed on a sample of that
// order's nodes; the faster route serves the order from then on.  Both routes
// satisfy the same residual gate, so the choice changes time, not the
// accuracy contract.
#include "labfm_internal.hpp"

#include <cstring>

namespace labfm {

void release_batch(Context* c) {
    if (c->batch.exec) hipGraphExecDestroy(c->batch.exec);
    c->batch.exec = nullptr;
    c->batch.sets.clear();
    c->batch.stream = nullptr;
}

namespace {

constexpr int64_t TUNE_SAMPLE = 4096;

bool same_opt(const labfm_wopts& a, const labfm_wopts& b) {
    return a.abf == b.abf && a.rbf == b.rbf && a.sigma == b.sigma && a.ops == b.ops && a.prec == b.prec &&
           a.tol_stop == b.tol_stop && a.tol_pass == b.tol_pass && a.max_iters == b.max_iters;
}

bool same_batch(const Context::Batch& b, int nsets, const labfm_node_set* sets, const labfm_wopts* opt,
                hipStream_t st) {
    return b.exec && b.stream == st && (int)b.sets.size() == nsets && same_opt(b.opt, *opt) &&
           memcmp(b.sets.data(), sets, sizeof(labfm_node_set) * (size_t)nsets) == 0;
}

NodeSet to_nodeset(const labfm_node_set& s) {
    NodeSet S{};
    S.x = s.x;
    S.y = s.y;
    S.R = s.R;
    S.order = s.order;
    S.row_ptr = s.row_ptr;
    S.col = s.col;
    S.n = s.n;
    S.nnz = s.nnz;
    S.Lx = s.dom.hi[0] - s.dom.lo[0];
    S.Ly = s.dom.hi[1] - s.dom.lo[1];
    S.perx = s.dom.periodic[0] != 0;
    S.pery = s.dom.periodic[1] != 0;
    S.w64 = s.w64;
    S.w32 = s.w32;
    S.status = s.status;
    S.resid = s.resid;
    S.iters = s.iters;
    S.psi0 = nullptr;
    return S;
}

Context::Tuned* find_tuned(Context* c, const WeightArgs& a, int K) {
    for (auto& t : c->tuned)
        if (t.abf == a.abf && t.rbf == a.rbf && t.ops == a.ops && t.order == K) return &t;
    return nullptr;
}

// Time both routes of every order present and not yet tuned; returns the
// orders routed to the FP64 kernels.
labfm_err tune(Context* c, const WeightArgs& a, const NodeSet* hs, int32_t* wl, int32_t* rl, int32_t* tcnt,
               hipStream_t st, unsigned* fp64_orders) {
    int32_t *list = wl, *off, *cnt;
    labfm_err e = build_order_lists(c, a, hs, st, &list, &off, &cnt);
    if (e != LABFM_OK) return e;
    int32_t hcnt[KMAX_ORDERS + 2];
    LABFM_HIP_CHECK(hipMemcpyAsync(hcnt, cnt, sizeof(hcnt), hipMemcpyDeviceToHost, st));
    LABFM_HIP_CHECK(hipStreamSynchronize(st));
    struct TimingOff {  // tuning launches are not reported as kernel timings
        Context* c;
        bool was;
        explicit TimingOff(Context* cc) : c(cc), was(cc->timing) { c->timing = false; }
        ~TimingOff() { c->timing = was; }
    } off_guard(c);
    unsigned mask = 0;
    for (int K = 1; K <= KMAX_ORDERS; ++K) {
        if (hcnt[K] <= 0) continue;
        Context::Tuned* t = find_tuned(c, a, K);
        if (!t) {
            const int64_t ns = hcnt[K] < TUNE_SAMPLE ? hcnt[K] : TUNE_SAMPLE;
            int32_t htc[KMAX_ORDERS + 2] = {};
            htc[K] = (int32_t)ns;
            LABFM_HIP_CHECK(hipMemcpyAsync(tcnt, htc, sizeof(htc), hipMemcpyHostToDevice, st));
            LABFM_HIP_CHECK(hipStreamSynchronize(st));
            hipEvent_t ev[3];
            for (auto& x : ev) LABFM_HIP_CHECK(hipEventCreate(&x));
            float ms_m = 0.f, ms_f = 0.f;
            for (int rep = 0; rep < 2; ++rep) {  // the first pass warms up
                LABFM_HIP_CHECK(hipEventRecord(ev[0], st));
                if ((e = weights_mixed_lists(c, a, list, off, tcnt, rl, 1u << K, st, 0, &c->batch.factors)) !=
                    LABFM_OK)
                    break;
                LABFM_HIP_CHECK(hipEventRecord(ev[1], st));
                if ((e = weights_fp64_split_lists(c, a, list, off, tcnt, 1u << K, c->batch.factors, st)) != LABFM_OK)
                    break;
                LABFM_HIP_CHECK(hipEventRecord(ev[2], st));
                LABFM_HIP_CHECK(hipEventSynchronize(ev[2]));
                LABFM_HIP_CHECK(hipEventElapsedTime(&ms_m, ev[0], ev[1]));
                LABFM_HIP_CHECK(hipEventElapsedTime(&ms_f, ev[1], ev[2]));
            }
            for (auto& x : ev) hipEventDestroy(x);
            if (e != LABFM_OK) return e;
            c->tuned.push_back({a.abf, a.rbf, a.ops, K, ms_f <= ms_m ? 2 : 1, (double)ms_m, (double)ms_f, ns});
            t = &c->tuned.back();
        }
        if (t->route == 2) mask |= 1u << K;
    }
    *fp64_orders = mask;
    return LABFM_OK;
}

labfm_err enqueue(Context* c, const WeightArgs& a, const NodeSet* hs, int32_t* wl, int32_t* rl, unsigned fp64_orders,
                  int prec, hipStream_t st) {
    return prec == LABFM_PREC_FP64 ? weights_fp64_split(c, a, hs, wl, c->batch.factors, st)
                                   : weights_mixed(c, a, hs, wl, rl, fp64_orders, st, 0, &c->batch.factors);
}

}  // namespace

labfm_err weights_batched(Context* c, int nsets, const labfm_node_set* sets, const labfm_wopts* opt, int use_graph,
                          hipStream_t st) {
    Context::Batch& B = c->batch;
    if (use_graph && same_batch(B, nsets, sets, opt, st)) {
        KernelTimer timer(c, "weights_batch_graph", st);
        LABFM_HIP_CHECK(hipGraphLaunch(B.exec, st));
        return LABFM_OK;
    }
    // a new plan: the previous graph (and the buffers it reads) is released first
    if (B.exec) LABFM_HIP_CHECK(hipStreamSynchronize(B.stream));
    LABFM_HIP_CHECK(hipStreamSynchronize(st));
    release_batch(c);
    std::vector<NodeSet> hs((size_t)nsets);
    std::vector<int64_t> hoff((size_t)nsets + 1, 0);
    for (int s = 0; s < nsets; ++s) {
        hs[s] = to_nodeset(sets[s]);
        hoff[s + 1] = hoff[s] + sets[s].n;
    }
    const int64_t ntotal = hoff[nsets];
    WeightArgs a{};
    set_options(a, opt);
    a.nsets = nsets;
    a.ntotal = ntotal;
    labfm_err e;
    if ((e = ensure(B.d_sets, sizeof(NodeSet) * (size_t)nsets)) != LABFM_OK) return e;
    if ((e = ensure(B.d_off, sizeof(int64_t) * (size_t)(nsets + 1))) != LABFM_OK) return e;
    if ((e = ensure(B.wl, sizeof(int32_t) * (size_t)(ntotal + 3 * (KMAX_ORDERS + 2)))) != LABFM_OK) return e;
    if ((e = ensure(B.rl, sizeof(int32_t) * (size_t)(ntotal + 2 * (KMAX_ORDERS + 2)))) != LABFM_OK) return e;
    LABFM_HIP_CHECK(hipMemcpyAsync(B.d_sets.p, hs.data(), sizeof(NodeSet) * (size_t)nsets, hipMemcpyHostToDevice, st));
    LABFM_HIP_CHECK(hipMemcpyAsync(B.d_off.p, hoff.data(), sizeof(int64_t) * (size_t)(nsets + 1),
                                   hipMemcpyHostToDevice, st));
    LABFM_HIP_CHECK(hipStreamSynchronize(st));
    a.sets = (const NodeSet*)B.d_sets.p;
    a.set_off = (const int64_t*)B.d_off.p;
    int32_t* wl = (int32_t*)B.wl.p;
    int32_t* rl = (int32_t*)B.rl.p;
    int32_t* tcnt = rl + ntotal + (KMAX_ORDERS + 2);  // tuning counters, after the retry list

    // the FP64 factor workspace and launch grids, sized here so that nothing allocates under capture
    if ((e = fp64_split_reserve(B.factors, ntotal)) != LABFM_OK) return e;
    init_split_grids();

    unsigned fp64_orders = 0;
    if (opt->prec == LABFM_PREC_MIXED)
        if ((e = tune(c, a, hs.data(), wl, rl, tcnt, st, &fp64_orders)) != LABFM_OK) return e;
    if (!use_graph) return enqueue(c, a, hs.data(), wl, rl, fp64_orders, opt->prec, st);

    init_weight_grids();
    init_mixed_grids();
    hipStream_t cap;
    LABFM_HIP_CHECK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        hipStreamDestroy(cap);
        set_error("labfm_weights_batched: hipStreamBeginCapture failed");
        return LABFM_EHIP;
    }
    e = enqueue(c, a, hs.data(), wl, rl, fp64_orders, opt->prec, cap);
    hipError_t he = hipStreamEndCapture(cap, &graph);
    hipGraphExec_t exec = nullptr;
    if (e == LABFM_OK && he == hipSuccess) he = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) hipGraphDestroy(graph);
    hipStreamDestroy(cap);
    if (e != LABFM_OK) return e;
    if (he != hipSuccess) {
        set_error(std::string("labfm_weights_batched: graph capture: ") + hipGetErrorString(he));
        return LABFM_EHIP;
    }
    B.exec = exec;
    B.stream = st;
    B.opt = *opt;
    B.opt.mlp = nullptr;
    B.sets.assign(sets, sets + nsets);
    B.fp64_orders = fp64_orders;
    KernelTimer timer(c, "weights_batch_graph", st);
    LABFM_HIP_CHECK(hipGraphLaunch(B.exec, st));
    return LABFM_OK;
}

labfm_err autotune_query(Context* c, int abf, int rbf, unsigned ops, int order, int* route, double* ms_mixed,
                         double* ms_fp64, int64_t* sample) {
    for (auto& t : c->tuned)
        if (t.abf == abf && t.rbf == rbf && t.ops == ops && t.order == order) {
            if (route) *route = t.route;
            if (ms_mixed) *ms_mixed = t.ms_mixed;
            if (ms_fp64) *ms_fp64 = t.ms_fp64;
            if (sample) *sample = t.sample;
            return LABFM_OK;
        }
    if (route) *route = 0;
    if (ms_mixed) *ms_mixed = 0.0;
    if (ms_fp64) *ms_fp64 = 0.0;
    if (sample) *sample = 0;
    return LABFM_OK;
}

}  // namespace labfm
