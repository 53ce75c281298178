// api.hip -- the extern "C" entry points declared in include/labfm.h:
// argument validation, context and scratch management, launch dispatch.
#include "labfm_internal.hpp"

#include <mutex>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>

namespace labfm {

namespace {
thread_local std::string g_last_error;

struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) hipSetDevice(prev);
    }
};

labfm_err fail(labfm_err e, const std::string& msg) {
    set_error(msg);
    return e;
}

GridSpec make_grid(const labfm_domain* d, int64_t n) {
    // about four nodes per bucket; the search visits ceil(R/w) rings
    GridSpec g{};
    g.Lx = d->hi[0] - d->lo[0];
    g.Ly = d->hi[1] - d->lo[1];
    double cells = (double)(n > 0 ? n : 1) / 4.0;
    double aspect = g.Lx / g.Ly;
    long ncx = lround(std::sqrt(cells * aspect));
    long ncy = lround(std::sqrt(cells / aspect));
    if (ncx < 1) ncx = 1;
    if (ncy < 1) ncy = 1;
    if (ncx > 8192) ncx = 8192;
    if (ncy > 8192) ncy = 8192;
    g.ncx = (int)ncx;
    g.ncy = (int)ncy;
    g.lox = d->lo[0];
    g.loy = d->lo[1];
    g.wx = g.Lx / g.ncx;
    g.wy = g.Ly / g.ncy;
    g.perx = d->periodic[0] != 0;
    g.pery = d->periodic[1] != 0;
    return g;
}

bool domain3_ok(const labfm_domain3* d) {
    if (!d) return false;
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(d->lo[a]) || !std::isfinite(d->hi[a]) || !(d->hi[a] > d->lo[a])) return false;
    return true;
}

Grid3 make_grid3(const labfm_domain3* d, int64_t n) {
    // about four nodes per bucket; the search visits ceil(R/w) cells each way
    Grid3 g{};
    double vol = 1.0;
    for (int a = 0; a < 3; ++a) {
        g.L[a] = d->hi[a] - d->lo[a];
        vol *= g.L[a];
    }
    const double per_len = std::cbrt((double)(n > 0 ? n : 1) / 4.0 / vol);
    for (int a = 0; a < 3; ++a) {
        long nc = lround(g.L[a] * per_len);
        if (nc < 1) nc = 1;
        if (nc > 256) nc = 256;
        g.nc[a] = (int)nc;
        g.lo[a] = d->lo[a];
        g.w[a] = g.L[a] / g.nc[a];
        g.per[a] = d->periodic[a] != 0;
    }
    return g;
}

int popcount5(unsigned ops) {
    int k = 0;
    for (int b = 0; b < 5; ++b) k += (ops >> b) & 1u;
    return k;
}

// structural checks of a network description (device pointers non-NULL, sizes in range)
bool mlp_ok(const labfm_mlp* net, std::string& why) {
    if (!net) return why = "network is NULL", false;
    if (net->n_layers < 1 || net->n_layers > LABFM_MLP_MAX_LAYERS) return why = "n_layers must be 1..8", false;
    for (int l = 0; l <= net->n_layers; ++l)
        if (net->dims[l] < 1 || net->dims[l] > 4096) return why = "layer widths must be 1..4096", false;
    for (int l = 0; l < net->n_layers; ++l)
        if (!net->W[l] || !net->b[l]) return why = "NULL weight or bias", false;
    return true;
}

// a network that serves the weight solve: features in, Psi of `ops` at `order` out
bool mlp_serves(const labfm_mlp* net, std::string& why) {
    if (!mlp_ok(net, why)) return false;
    if (net->kmax < 1 || net->kmax > LABFM_MAX_NEIGHBOURS) return why = "kmax must be 1..128", false;
    if (net->dims[0] != 3 * net->kmax) return why = "dims[0] must be 3 kmax", false;
    if (net->order < 1 || net->order > LABFM_MAX_ORDER) return why = "order must be 1..8", false;
    if (net->ops == 0 || (net->ops & ~31u)) return why = "bad ops", false;
    const int p = (net->order * net->order + 3 * net->order) / 2;
    if (net->dims[net->n_layers] != popcount5(net->ops) * p) return why = "output width must be nops * p(order)", false;
    if (!net->mu || !net->sd) return why = "mu and sd are required", false;
    return true;
}

bool domain_ok(const labfm_domain* d) {
    return d && std::isfinite(d->lo[0]) && std::isfinite(d->lo[1]) && std::isfinite(d->hi[0]) &&
           std::isfinite(d->hi[1]) && d->hi[0] > d->lo[0] && d->hi[1] > d->lo[1];
}

}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

// options shared by every node set of a weight computation
void set_options(WeightArgs& a, const labfm_wopts* opt) {
    a.abf = opt->abf;
    a.rbf = opt->rbf;
    a.sigma = opt->sigma;
    a.ops = opt->ops;
    a.nops = popcount5(opt->ops);
    a.tol_stop = opt->tol_stop;
    a.tol_pass = opt->tol_pass;
    a.max_iters = opt->max_iters;
    a.iters_offset = 0;
    a.max_iters32 = 30;
    a.psi0_order = 0;
    a.psi0_ld = 0;
}


labfm_err ensure(Scratch& s, size_t bytes) {
    if (bytes == 0) bytes = 1;
    if (s.bytes >= bytes) return LABFM_OK;
    if (s.p) hipFree(s.p);
    s.p = nullptr;
    s.bytes = 0;
    size_t want = bytes + bytes / 4;
    if (hipMalloc(&s.p, want) != hipSuccess) {
        s.p = nullptr;
        set_error("scratch allocation of " + std::to_string(want) + " bytes failed");
        return LABFM_ENOMEM;
    }
    s.bytes = want;
    return LABFM_OK;
}

}  // namespace labfm

using namespace labfm;

extern "C" {

const char* labfm_last_error(void) { return g_last_error.c_str(); }

namespace {
labfm_err scratch_setup(int device);
}

labfm_err labfm_create(void** ctx, int device) {
    if (!ctx) return fail(LABFM_EINVAL, "labfm_create: ctx is NULL");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(LABFM_EHIP, "labfm_create: no HIP device");
    if (device < 0 || device >= ndev) return fail(LABFM_EINVAL, "labfm_create: bad device id");
    labfm_err e = scratch_setup(device);
    if (e != LABFM_OK) return e;
    Context* c = new Context();
    c->device = device;
    *ctx = c;
    return LABFM_OK;
}

labfm_err labfm_destroy(void* ctx) {
    if (!ctx) return LABFM_OK;
    Context* c = (Context*)ctx;
    DeviceGuard g(c->device);
    if (c->step_exec) hipStreamSynchronize(c->step_stream);
    release_step_graph(c);
    if (c->burgers.exec) hipStreamSynchronize(c->burgers.stream);
    release_burgers_graph(c);
    if (c->batch.exec) hipStreamSynchronize(c->batch.stream);
    release_batch(c);
    for (auto& t : c->timed) {
        hipEventDestroy(t.a);
        hipEventDestroy(t.b);
    }
    Scratch* all[] = {&c->grid_count, &c->grid_idx, &c->node_cell, &c->counts, &c->scan_tmp, &c->worklist,
                      &c->mixed,      &c->mlp_act,  &c->mlp_feat,  &c->mlp_psi, &c->mlp_part, &c->poisson,
                      &c->factors, &c->factors3,
                      &c->batch.d_sets, &c->batch.d_off, &c->batch.wl, &c->batch.rl, &c->batch.factors};
    for (Scratch* s : all)
        if (s->p) hipFree(s->p);
    delete c;
    return LABFM_OK;
}

labfm_err labfm_build_neighbours(void* ctx, const double* x, const double* y, int64_t n, const labfm_domain* dom,
                                 double* R, const int8_t* order, int grow, int max_grow, int64_t* row_ptr,
                                 int32_t* col, int64_t* nnz_host, void* stream) {
    if (!ctx) return fail(LABFM_EINVAL, "labfm_build_neighbours: ctx is NULL");
    if (n < 0 || n > INT32_MAX) return fail(LABFM_EINVAL, "labfm_build_neighbours: n out of range [0, 2^31)");
    if (!domain_ok(dom)) return fail(LABFM_EINVAL, "labfm_build_neighbours: bad domain");
    if (n > 0 && (!x || !y || !R || !row_ptr)) return fail(LABFM_EINVAL, "labfm_build_neighbours: NULL array");
    if (!col && grow && n > 0 && !order) return fail(LABFM_EINVAL, "labfm_build_neighbours: order needed to grow");
    if (max_grow < 0 || max_grow > 64) return fail(LABFM_EINVAL, "labfm_build_neighbours: max_grow out of range");
    if (!col && !nnz_host) return fail(LABFM_EINVAL, "labfm_build_neighbours: nnz_host is NULL on the count pass");
    Context* c = (Context*)ctx;
    DeviceGuard g(c->device);
    if (!g.ok) return fail(LABFM_EHIP, "labfm_build_neighbours: hipSetDevice failed");
    hipStream_t st = (hipStream_t)stream;
    GridSpec grid = make_grid(dom, n);
    if (!col) {
        labfm_err e = n > 0 ? neighbours_count(c, x, y, n, grid, R, order, grow, max_grow, row_ptr, st)
                            : exclusive_scan_i64(c, nullptr, row_ptr, 0, st);
        if (e != LABFM_OK) return e;
        LABFM_HIP_CHECK(hipMemcpyAsync(nnz_host, row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        LABFM_HIP_CHECK(hipStreamSynchronize(st));
        return LABFM_OK;
    }
    if (n == 0) return LABFM_OK;
    return neighbours_fill(c, x, y, n, grid, R, row_ptr, col, st);
}

labfm_err labfm_build_neighbours3(void* ctx, const double* x, const double* y, const double* z, int64_t n,
                                  const labfm_domain3* dom, const double* R, int64_t* row_ptr, int32_t* col,
                                  int64_t* nnz_host, void* stream) {
    if (!ctx) return fail(LABFM_EINVAL, "labfm_build_neighbours3: ctx is NULL");
    if (n < 0 || n > INT32_MAX) return fail(LABFM_EINVAL, "labfm_build_neighbours3: n out of range [0, 2^31)");
    if (!domain3_ok(dom)) return fail(LABFM_EINVAL, "labfm_build_neighbours3: bad domain");
    if (n > 0 && (!x || !y || !z || !R || !row_ptr)) return fail(LABFM_EINVAL, "labfm_build_neighbours3: NULL array");
    if (!col && !nnz_host) return fail(LABFM_EINVAL, "labfm_build_neighbours3: nnz_host is NULL on the count pass");
    Context* c = (Context*)ctx;
    DeviceGuard g(c->device);
    if (!g.ok) return fail(LABFM_EHIP, "labfm_build_neighbours3: hipSetDevice failed");
    hipStream_t st = (hipStream_t)stream;
    Grid3 grid = make_grid3(dom, n);
    if (!col) {
        labfm_err e = n > 0 ? neighbours3_count(c, x, y, z, n, grid, R, row_ptr, st)
                            : exclusive_scan_i64(c, nullptr, row_ptr, 0, st);
        if (e != LABFM_OK) return e;
        LABFM_HIP_CHECK(hipMemcpyAsync(nnz_host, row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        LABFM_HIP_CHECK(hipStreamSynchronize(st));
        return LABFM_OK;
    }
    if (n == 0) return LABFM_OK;
    return neighbours3_fill(c, x, y, z, n, grid, R, row_ptr, col, st);
}

labfm_err labfm_weights3(void* ctx, const double* x, const double* y, const double* z, int64_t n,
                         const labfm_domain3* dom, const double* R, int k, const int64_t* row_ptr,
                         const int32_t* col, int64_t nnz, const labfm_wopts* opt, double* w64, int8_t* status,
                         float* resid, int8_t* iters, void* stream) {
    if (!ctx) return fail(LABFM_EINVAL, "labfm_weights3: ctx is NULL");
    if (!opt) return fail(LABFM_EINVAL, "labfm_weights3: opt is NULL");
    if (n < 0 || n > INT32_MAX || nnz < 0) return fail(LABFM_EINVAL, "labfm_weights3: n or nnz out of range");
    if (!domain3_ok(dom)) return fail(LABFM_EINVAL, "labfm_weights3: bad domain");
    if (k < 1 || k > LABFM_MAX_ORDER3) return fail(LABFM_EINVAL, "labfm_weights3: k must be 1..6");
    const unsigned allowed = LABFM_OP_DX | LABFM_OP_DY | LABFM_OP_LAP | LABFM_OP_DZ;
    if (opt->ops == 0 || (opt->ops & ~allowed))
        return fail(LABFM_EINVAL, "labfm_weights3: ops must be a nonzero set of DX, DY, DZ, LAP");
    if (opt->abf != LABFM_ABF_HERMITE) return fail(LABFM_EUNSUPPORTED, "labfm_weights3: only the HERMITE family");
    if (opt->prec != LABFM_PREC_FP64) return fail(LABFM_EUNSUPPORTED, "labfm_weights3: only LABFM_PREC_FP64");
    if (opt->rbf < 0 || opt->rbf > 4) return fail(LABFM_EINVAL, "labfm_weights3: bad rbf");
    if (!(opt->sigma > 0.0) || !std::isfinite(opt->sigma)) return fail(LABFM_EINVAL, "labfm_weights3: sigma must be > 0");
    if (opt->max_iters < 0 || opt->max_iters > 63) return fail(LABFM_EINVAL, "labfm_weights3: max_iters must be in 0..63");
    if (!(opt->tol_stop >= 0.0) || !(opt->tol_pass >= 0.0)) return fail(LABFM_EINVAL, "labfm_weights3: bad tolerances");
    if (n > 0 && (!x || !y || !z || !R || !row_ptr || !status || !w64 || (nnz > 0 && !col)))
        return fail(LABFM_EINVAL, "labfm_weights3: NULL array");
    Context* c = (Context*)ctx;
    DeviceGuard g(c->device);
    if (!g.ok) return fail(LABFM_EHIP, "labfm_weights3: hipSetDevice failed");
    return weights3(c, x, y, z, n, make_grid3(dom, n), R, k, row_ptr, col, nnz, opt, w64, status, resid, iters,
                    (hipStream_t)stream);
}

namespace {

// Argument checks shared by labfm_weights and labfm_weights_noalloc (`who`
// prefixes the message), and the WeightArgs of the call's one node set.
labfm_err check_weights_args(const char* who, const double* x, const double* y, int64_t n, const labfm_domain* dom,
                             const double* R, const int8_t* order, const int64_t* row_ptr, const int32_t* col,
                             int64_t nnz, const labfm_wopts* opt, double* w64, float* w32, int8_t* status) {
    const std::string w = std::string(who) + ": ";
    if (!opt) return fail(LABFM_EINVAL, w + "opt is NULL");
    if (n < 0 || n > INT32_MAX || nnz < 0) return fail(LABFM_EINVAL, w + "n or nnz out of range");
    if (!domain_ok(dom)) return fail(LABFM_EINVAL, w + "bad domain");
    if (opt->ops == 0 || (opt->ops & ~31u)) return fail(LABFM_EINVAL, w + "ops must be a nonzero set of LABFM_OP_* bits");
    if (opt->abf < LABFM_ABF_HERMITE || opt->abf > LABFM_ABF_PAPER_D1) return fail(LABFM_EINVAL, w + "bad abf");
    if (opt->rbf < 0 || opt->rbf > 4) return fail(LABFM_EINVAL, w + "bad rbf");
    if (!(opt->sigma > 0.0) || !std::isfinite(opt->sigma)) return fail(LABFM_EINVAL, w + "sigma must be > 0");
    if (opt->max_iters < 0 || opt->max_iters > 63) return fail(LABFM_EINVAL, w + "max_iters must be in 0..63");
    if (!(opt->tol_stop >= 0.0) || !(opt->tol_pass >= 0.0)) return fail(LABFM_EINVAL, w + "bad tolerances");
    if (!w64 && !w32) return fail(LABFM_EINVAL, w + "w64 and w32 are both NULL");
    if (n > 0 && (!x || !y || !R || !order || !row_ptr || !status || (nnz > 0 && !col)))
        return fail(LABFM_EINVAL, w + "NULL array");
    if (opt->prec != LABFM_PREC_FP64 && opt->prec != LABFM_PREC_MIXED && opt->prec != LABFM_PREC_MLP &&
        opt->prec != LABFM_PREC_MLP_NOLU)
        return fail(LABFM_EINVAL, w + "bad prec");
    return LABFM_OK;
}

void one_set_args(WeightArgs& a, const double* x, const double* y, int64_t n, const labfm_domain* dom,
                  const double* R, const int8_t* order, const int64_t* row_ptr, const int32_t* col, int64_t nnz,
                  const labfm_wopts* opt, double* w64, float* w32, int8_t* status, float* resid, int8_t* iters) {
    a = WeightArgs{};
    NodeSet& S = a.one;
    S.x = x;
    S.y = y;
    S.R = R;
    S.order = order;
    S.row_ptr = row_ptr;
    S.col = col;
    S.n = n;
    S.nnz = nnz;
    S.Lx = dom->hi[0] - dom->lo[0];
    S.Ly = dom->hi[1] - dom->lo[1];
    S.perx = dom->periodic[0] != 0;
    S.pery = dom->periodic[1] != 0;
    S.w64 = w64;
    S.w32 = w32;
    S.status = status;
    S.resid = resid;
    S.iters = iters;
    S.psi0 = nullptr;
    a.sets = nullptr;
    a.set_off = nullptr;
    a.nsets = 1;
    a.ntotal = n;
    set_options(a, opt);
}

// ---- the weights entry point that allocates nothing -----------------------
// Its work lists (n + 3 (KMAX + 2) int32) and the mixed path's retry list
// (n + KMAX + 2 int32) live in this file-scope array, one copy per GPU, held
// until the process ends.  Host code never passes the array's name to a
// kernel: each device's address comes from hipGetSymbolAddress, taken once
// per device in labfm_create with that device current.
constexpr int64_t NOALLOC_MAX_NODES = LABFM_NOALLOC_MAX_NODES;
constexpr int64_t NOALLOC_WL_INTS = NOALLOC_MAX_NODES + 3 * (LABFM_MAX_ORDER + 2);
constexpr int64_t NOALLOC_RL_INTS = NOALLOC_MAX_NODES + (LABFM_MAX_ORDER + 2);
static __device__ __align__(256) int32_t scratch[NOALLOC_WL_INTS + NOALLOC_RL_INTS];
constexpr int NOALLOC_MAX_DEVICES = 64;
int32_t* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};
std::mutex g_scratch_mu;

labfm_err scratch_setup(int device) {
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return fail(LABFM_EINVAL, "labfm_create: device id above 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return LABFM_OK;
    DeviceGuard g(device);
    if (!g.ok) return fail(LABFM_EHIP, "labfm_create: hipSetDevice failed");
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(LABFM_EHIP, std::string("labfm_create: hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = (int32_t*)p;
    return LABFM_OK;
}

}  // namespace

labfm_err labfm_weights(void* ctx, const double* x, const double* y, int64_t n, const labfm_domain* dom,
                        const double* R, const int8_t* order, const int64_t* row_ptr, const int32_t* col,
                        int64_t nnz, const labfm_wopts* opt, double* w64, float* w32, int8_t* status, float* resid,
                        int8_t* iters, void* stream) {
    if (!ctx) return fail(LABFM_EINVAL, "labfm_weights: ctx is NULL");
    labfm_err e = check_weights_args("labfm_weights", x, y, n, dom, R, order, row_ptr, col, nnz, opt, w64, w32, status);
    if (e != LABFM_OK) return e;
    if (opt->prec == LABFM_PREC_MLP || opt->prec == LABFM_PREC_MLP_NOLU) {
        std::string why;
        if (!mlp_serves(opt->mlp, why)) return fail(LABFM_EINVAL, "labfm_weights: network: " + why);
        if (opt->mlp->ops != opt->ops) return fail(LABFM_EINVAL, "labfm_weights: network ops differ from opt->ops");
    }
    Context* c = (Context*)ctx;
    DeviceGuard g(c->device);
    if (!g.ok) return fail(LABFM_EHIP, "labfm_weights: hipSetDevice failed");
    if (n == 0) return LABFM_OK;
    WeightArgs a;
    one_set_args(a, x, y, n, dom, R, order, row_ptr, col, nnz, opt, w64, w32, status, resid, iters);
    hipStream_t st = (hipStream_t)stream;
    if ((e = ensure(c->worklist, sizeof(int32_t) * (size_t)(n + 3 * (LABFM_MAX_ORDER + 2)))) != LABFM_OK) return e;
    int32_t* wl = (int32_t*)c->worklist.p;
    if (opt->prec == LABFM_PREC_FP64) return weights_fp64_split(c, a, &a.one, wl, c->factors, st);
    if ((e = ensure(c->mixed, sizeof(int32_t) * (size_t)(n + LABFM_MAX_ORDER + 2))) != LABFM_OK) return e;
    int32_t* rl = (int32_t*)c->mixed.p;
    if (opt->prec == LABFM_PREC_MIXED) return weights_mixed(c, a, &a.one, wl, rl, 0u, st, 0, &c->factors);
    return weights_mlp(c, a, wl, rl, opt->mlp, st, opt->prec == LABFM_PREC_MLP_NOLU);
}

labfm_err labfm_weights_noalloc(void* ctx, const double* x, const double* y, int64_t n, const labfm_domain* dom,
                                const double* R, const int8_t* order, const int64_t* row_ptr, const int32_t* col,
                                int64_t nnz, const labfm_wopts* opt, double* w64, float* w32, int8_t* status,
                                float* resid, int8_t* iters, void* stream) {
    if (!ctx) return fail(LABFM_EINVAL, "labfm_weights_noalloc: ctx is NULL");
    labfm_err e =
        check_weights_args("labfm_weights_noalloc", x, y, n, dom, R, order, row_ptr, col, nnz, opt, w64, w32, status);
    if (e != LABFM_OK) return e;
    if (opt->prec == LABFM_PREC_MLP || opt->prec == LABFM_PREC_MLP_NOLU)
        return fail(LABFM_EUNSUPPORTED, "labfm_weights_noalloc: the warm start needs library scratch; use labfm_weights");
    if (n > NOALLOC_MAX_NODES)
        return fail(LABFM_EINVAL, "labfm_weights_noalloc: n = " + std::to_string(n) + " exceeds LABFM_NOALLOC_MAX_NODES (" +
                                      std::to_string(NOALLOC_MAX_NODES) + ")");
    Context* c = (Context*)ctx;
    int32_t* base = (c->device >= 0 && c->device < NOALLOC_MAX_DEVICES) ? g_scratch_ptr[c->device] : nullptr;
    if (!base) return fail(LABFM_EINVAL, "labfm_weights_noalloc: no scratch address for this device (context not from labfm_create)");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(LABFM_EHIP, "labfm_weights_noalloc: hipSetDevice failed");
    if (n == 0) return LABFM_OK;
    WeightArgs a;
    one_set_args(a, x, y, n, dom, R, order, row_ptr, col, nnz, opt, w64, w32, status, resid, iters);
    // kernel timing records HIP events, which this entry point does not create
    struct TimingOff {
        Context* c;
        bool was;
        explicit TimingOff(Context* cc) : c(cc), was(cc->timing) { c->timing = false; }
        ~TimingOff() { c->timing = was; }
    } off(c);
    hipStream_t st = (hipStream_t)stream;
    int32_t* wl = base;                    // work lists: counters are cleared by a kernel inside
    int32_t* rl = base + NOALLOC_WL_INTS;  // retry list of the mixed path: the same
    if (opt->prec == LABFM_PREC_FP64) return weights_fp64(c, a, &a.one, wl, st);
    return weights_mixed(c, a, &a.one, wl, rl, 0u, st);
}

labfm_err labfm_weights_batched(void* ctx, int nsets, const labfm_node_set* sets, const labfm_wopts* opt,
                                int use_graph, void* stream) {
    if (!ctx || !opt) return fail(LABFM_EINVAL, "labfm_weights_batched: ctx or opt is NULL");
    if (nsets < 1 || !sets) return fail(LABFM_EINVAL, "labfm_weights_batched: need nsets >= 1 and a set table");
    if (opt->ops == 0 || (opt->ops & ~31u)) return fail(LABFM_EINVAL, "labfm_weights_batched: bad ops");
    if (opt->abf < LABFM_ABF_HERMITE || opt->abf > LABFM_ABF_PAPER_D1) return fail(LABFM_EINVAL, "labfm_weights_batched: bad abf");
    if (opt->rbf < 0 || opt->rbf > 4) return fail(LABFM_EINVAL, "labfm_weights_batched: bad rbf");
    if (!(opt->sigma > 0.0) || !std::isfinite(opt->sigma)) return fail(LABFM_EINVAL, "labfm_weights_batched: sigma must be > 0");
    if (opt->max_iters < 0 || opt->max_iters > 63) return fail(LABFM_EINVAL, "labfm_weights_batched: max_iters must be in 0..63");
    if (!(opt->tol_stop >= 0.0) || !(opt->tol_pass >= 0.0)) return fail(LABFM_EINVAL, "labfm_weights_batched: bad tolerances");
    if (opt->prec == LABFM_PREC_MLP || opt->prec == LABFM_PREC_MLP_NOLU)
        return fail(LABFM_EUNSUPPORTED, "labfm_weights_batched: the warm start is not batched");
    if (opt->prec != LABFM_PREC_FP64 && opt->prec != LABFM_PREC_MIXED) return fail(LABFM_EINVAL, "labfm_weights_batched: bad prec");
    int64_t total = 0;
    for (int s = 0; s < nsets; ++s) {
        const labfm_node_set& S = sets[s];
        const std::string where = "labfm_weights_batched: set " + std::to_string(s) + ": ";
        if (S.n < 0 || S.nnz < 0) return fail(LABFM_EINVAL, where + "negative size");
        if (!domain_ok(&S.dom)) return fail(LABFM_EINVAL, where + "bad domain");
        if (!S.w64 && !S.w32) return fail(LABFM_EINVAL, where + "w64 and w32 are both NULL");
        if (S.n > 0 && (!S.x || !S.y || !S.R || !S.order || !S.row_ptr || !S.status || (S.nnz > 0 && !S.col)))
            return fail(LABFM_EINVAL, where + "NULL array");
        total += S.n;
    }
    if (total > INT32_MAX - 64) return fail(LABFM_EINVAL, "labfm_weights_batched: more than 2^31 nodes in total");
    Context* c = (Context*)ctx;
    DeviceGuard g(c->device);
    if (total == 0) return LABFM_OK;
    return weights_batched(c, nsets, sets, opt, use_graph, (hipStream_t)stream);
}

labfm_err labfm_autotune_query(void* ctx, int abf, int rbf, unsigned ops, int order, int* route, double* ms_mixed,
                               double* ms_fp64, int64_t* sample) {
    if (!ctx) return fail(LABFM_EINVAL, "labfm_autotune_query: ctx is NULL");
    return autotune_query((Context*)ctx, abf, rbf, ops, order, route, ms_mixed, ms_fp64, sample);
}

labfm_err labfm_combine(void* ctx, const double* w64, int nsets, const double* coef, int64_t nnz, double* out64,
                        float* out32, void* stream) {
    if (!ctx) return fail(LABFM_EINVAL, "labfm_combine: ctx is NULL");
    if (nsets < 1 || nsets > 5) return fail(LABFM_EINVAL, "labfm_combine: nsets must be 1..5");
    if (nnz < 0) return fail(LABFM_EINVAL, "labfm_combine: nnz < 0");
    if (!coef || (nnz > 0 && !w64) || (!out64 && !out32)) return fail(LABFM_EINVAL, "labfm_combine: NULL argument");
    Context* c = (Context*)ctx;
    DeviceGuard g(c->device);
    return combine_launch(w64, nsets, coef, nnz, out64, out32, (hipStream_t)stream);
}

labfm_err labfm_apply_operator(void* ctx, const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t nnz,
                               int nops, const void* w, int dtype, const void* u, void* out, void* stream) {
    if (!ctx) return fail(LABFM_EINVAL, "labfm_apply_operator: ctx is NULL");
    if (n < 0 || nnz < 0) return fail(LABFM_EINVAL, "labfm_apply_operator: n or nnz < 0");
    if (nops < 1 || nops > 5) return fail(LABFM_EINVAL, "labfm_apply_operator: nops must be 1..5");
    if (dtype != 0 && dtype != 1) return fail(LABFM_EINVAL, "labfm_apply_operator: dtype must be 0 (FP32) or 1 (FP64)");
    if (n > 0 && (!row_ptr || !u || !out || (nnz > 0 && (!col || !w))))
        return fail(LABFM_EINVAL, "labfm_apply_operator: NULL array");
    Context* c = (Context*)ctx;
    DeviceGuard g(c->device);
    return apply_launch(c, row_ptr, col, n, nnz, nops, w, dtype, u, out, (hipStream_t)stream);
}

labfm_err labfm_step(void* ctx, const labfm_step_plan* plan, void* u, void* scratch, int nsteps, int use_graph,
                     void* stream) {
    if (!ctx || !plan) return fail(LABFM_EINVAL, "labfm_step: ctx or plan is NULL");
    if (plan->n < 0 || plan->nnz < 0 || nsteps < 0) return fail(LABFM_EINVAL, "labfm_step: negative size");
    if (plan->dtype != 0 && plan->dtype != 1) return fail(LABFM_EINVAL, "labfm_step: dtype must be 0 or 1");
    if (plan->n > 0 && (!plan->row_ptr || !u || !scratch || (plan->nnz > 0 && (!plan->col || !plan->w_lin))))
        return fail(LABFM_EINVAL, "labfm_step: NULL array");
    if (!std::isfinite(plan->dt) || !std::isfinite(plan->gamma)) return fail(LABFM_EINVAL, "labfm_step: dt/gamma not finite");
    Context* c = (Context*)ctx;
    DeviceGuard g(c->device);
    return step_launch(c, plan, u, scratch, nsteps, use_graph, (hipStream_t)stream);
}

labfm_err labfm_burgers_step(void* ctx, const labfm_burgers_plan* plan, void* u, void* v, void* scratch, int nsteps,
                             int use_graph, void* stream) {
    if (!ctx || !plan) return fail(LABFM_EINVAL, "labfm_burgers_step: ctx or plan is NULL");
    if (plan->n < 0 || plan->nnz < 0 || nsteps < 0) return fail(LABFM_EINVAL, "labfm_burgers_step: negative size");
    if (plan->dtype != 0 && plan->dtype != 1) return fail(LABFM_EINVAL, "labfm_burgers_step: dtype must be 0 or 1");
    if (plan->n > 0 && (!plan->row_ptr || !u || !v || !scratch ||
                        (plan->nnz > 0 && (!plan->col || !plan->w_x || !plan->w_y || !plan->w_lap))))
        return fail(LABFM_EINVAL, "labfm_burgers_step: NULL array");
    if (plan->n > 0 && (u == v || u == scratch || v == scratch))
        return fail(LABFM_EINVAL, "labfm_burgers_step: u, v and scratch must be distinct buffers");
    if (!std::isfinite(plan->dt) || !std::isfinite(plan->nu))
        return fail(LABFM_EINVAL, "labfm_burgers_step: dt/nu not finite");
    if (plan->dfix && !plan->fixed)
        return fail(LABFM_EINVAL, "labfm_burgers_step: dfix needs a fixed mask");
    if (plan->n > 0 && (uintptr_t)scratch % (plan->dtype ? 16 : 8) != 0)
        return fail(LABFM_EINVAL, "labfm_burgers_step: scratch must be aligned to two elements");
    Context* c = (Context*)ctx;
    DeviceGuard g(c->device);
    return burgers_launch(c, plan, u, v, scratch, nsteps, use_graph, (hipStream_t)stream);
}

labfm_err labfm_poisson_solve(void* ctx, const labfm_poisson_plan* plan, const double* F, double* phi, void* scratch,
                              int* iters, double* rel_resid, int* converged, void* stream) {
    if (!ctx || !plan) return fail(LABFM_EINVAL, "labfm_poisson_solve: ctx or plan is NULL");
    if (plan->n < 0 || plan->nnz < 0) return fail(LABFM_EINVAL, "labfm_poisson_solve: negative size");
    if (!(plan->tol > 0.0) || !std::isfinite(plan->tol)) return fail(LABFM_EINVAL, "labfm_poisson_solve: tol must be > 0");
    if (plan->max_iters < 0 || plan->check_every < 1)
        return fail(LABFM_EINVAL, "labfm_poisson_solve: max_iters >= 0 and check_every >= 1 required");
    if (plan->n > 0 && (!plan->row_ptr || !F || !phi || !scratch || (plan->nnz > 0 && (!plan->col || !plan->w_lap))))
        return fail(LABFM_EINVAL, "labfm_poisson_solve: NULL array");
    if (iters) *iters = 0;
    if (rel_resid) *rel_resid = 0.0;
    if (converged) *converged = 1;
    if (plan->n == 0) return LABFM_OK;
    Context* c = (Context*)ctx;
    DeviceGuard g(c->device);
    return poisson_solve(c, plan, F, phi, (double*)scratch, iters, rel_resid, converged, (hipStream_t)stream);
}

labfm_err labfm_neumann_rows(void* ctx, const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t nnz,
                             const double* w_x, const double* w_y, const double* w_lap, const int32_t* parent,
                             const double* nx, const double* ny, int64_t* out_row_ptr, int32_t* out_col,
                             double* out_w, int32_t* out_center, int64_t* nnz_host, void* stream) {
    if (!ctx) return fail(LABFM_EINVAL, "labfm_neumann_rows: ctx is NULL");
    if (n < 0 || nnz < 0 || n > INT32_MAX) return fail(LABFM_EINVAL, "labfm_neumann_rows: n or nnz out of range");
    if (!out_col && !nnz_host) return fail(LABFM_EINVAL, "labfm_neumann_rows: count pass needs nnz_host");
    if (out_col && (!out_w || !out_center)) return fail(LABFM_EINVAL, "labfm_neumann_rows: fill pass needs out_w and out_center");
    if (n > 0 && (!row_ptr || !out_row_ptr || (nnz > 0 && (!col || !w_x || !w_y || !w_lap)) || (parent && (!nx || !ny))))
        return fail(LABFM_EINVAL, "labfm_neumann_rows: NULL array");
    Context* c = (Context*)ctx;
    DeviceGuard g(c->device);
    if (!g.ok) return fail(LABFM_EHIP, "labfm_neumann_rows: hipSetDevice failed");
    hipStream_t st = (hipStream_t)stream;
    if (n == 0) {
        if (!out_col) {
            labfm_err e = exclusive_scan_i64(c, nullptr, out_row_ptr, 0, st);
            if (e != LABFM_OK) return e;
            *nnz_host = 0;
            LABFM_HIP_CHECK(hipStreamSynchronize(st));
        }
        return LABFM_OK;
    }
    return neumann_rows(c, row_ptr, col, n, w_x, w_y, w_lap, parent, nx, ny, out_row_ptr, out_col, out_w, out_center,
                        nnz_host, st);
}

labfm_err labfm_ns_step(void* ctx, const labfm_ns_plan* plan, double* omega, double* psi, void* scratch, int nsteps,
                        int* solver_iters, int* all_converged, void* stream) {
    if (!ctx || !plan) return fail(LABFM_EINVAL, "labfm_ns_step: ctx or plan is NULL");
    if (plan->n < 0 || plan->nnz < 0 || nsteps < 0) return fail(LABFM_EINVAL, "labfm_ns_step: negative size");
    if (!(plan->tol > 0.0) || !std::isfinite(plan->tol) || plan->max_iters < 0 || plan->check_every < 1)
        return fail(LABFM_EINVAL, "labfm_ns_step: tol > 0, max_iters >= 0 and check_every >= 1 required");
    if (!std::isfinite(plan->dt) || !std::isfinite(plan->nu)) return fail(LABFM_EINVAL, "labfm_ns_step: dt/nu not finite");
    if (plan->n > 0 && (!plan->row_ptr || !omega || !psi || !scratch ||
                        (plan->nnz > 0 && (!plan->col || !plan->w_x || !plan->w_y || !plan->w_lap))))
        return fail(LABFM_EINVAL, "labfm_ns_step: NULL array");
    if (plan->n > 0 && (omega == psi || (void*)omega == scratch || (void*)psi == scratch))
        return fail(LABFM_EINVAL, "labfm_ns_step: omega, psi and scratch must be distinct buffers");
    if (solver_iters) *solver_iters = 0;
    if (all_converged) *all_converged = 1;
    if (plan->n == 0 || nsteps == 0) return LABFM_OK;
    Context* c = (Context*)ctx;
    DeviceGuard g(c->device);
    return ns_step(c, plan, omega, psi, (double*)scratch, nsteps, solver_iters, all_converged, (hipStream_t)stream);
}

labfm_err labfm_mlp_features(void* ctx, const double* x, const double* y, int64_t n, const labfm_domain* dom,
                             const double* R, const int64_t* row_ptr, const int32_t* col, int kmax, float* feat,
                             void* stream) {
    if (!ctx) return fail(LABFM_EINVAL, "labfm_mlp_features: ctx is NULL");
    if (n < 0 || n > INT32_MAX) return fail(LABFM_EINVAL, "labfm_mlp_features: n out of range");
    if (kmax < 1 || kmax > LABFM_MAX_NEIGHBOURS) return fail(LABFM_EINVAL, "labfm_mlp_features: kmax must be 1..128");
    if (!domain_ok(dom)) return fail(LABFM_EINVAL, "labfm_mlp_features: bad domain");
    if (n > 0 && (!x || !y || !R || !row_ptr || !col || !feat)) return fail(LABFM_EINVAL, "labfm_mlp_features: NULL array");
    Context* c = (Context*)ctx;
    DeviceGuard g(c->device);
    return mlp_features(c, x, y, R, row_ptr, col, 0, n, dom->hi[0] - dom->lo[0], dom->hi[1] - dom->lo[1],
                        dom->periodic[0] != 0, dom->periodic[1] != 0, kmax, feat, (hipStream_t)stream);
}

labfm_err labfm_moment_systems(void* ctx, const double* x, const double* y, int64_t n, const labfm_domain* dom,
                               const double* R, int k, const int64_t* row_ptr, const int32_t* col, int64_t nnz,
                               const labfm_wopts* opt, float* M, float* psi, int8_t* status, void* stream) {
    if (!ctx || !opt) return fail(LABFM_EINVAL, "labfm_moment_systems: ctx or opt is NULL");
    if (n < 0 || n > INT32_MAX || nnz < 0) return fail(LABFM_EINVAL, "labfm_moment_systems: n or nnz out of range");
    if (k < 1 || k > LABFM_MAX_ORDER) return fail(LABFM_EINVAL, "labfm_moment_systems: k must be 1..8");
    if (!domain_ok(dom)) return fail(LABFM_EINVAL, "labfm_moment_systems: bad domain");
    if (opt->ops == 0 || (opt->ops & ~31u)) return fail(LABFM_EINVAL, "labfm_moment_systems: bad ops");
    if (opt->abf < LABFM_ABF_HERMITE || opt->abf > LABFM_ABF_PAPER_D1) return fail(LABFM_EINVAL, "labfm_moment_systems: bad abf");
    if (opt->rbf < 0 || opt->rbf > 4) return fail(LABFM_EINVAL, "labfm_moment_systems: bad rbf");
    if (!(opt->sigma > 0.0) || !std::isfinite(opt->sigma)) return fail(LABFM_EINVAL, "labfm_moment_systems: sigma must be > 0");
    if (n > 0 && (!x || !y || !R || !row_ptr || !M || !psi || !status || (nnz > 0 && !col)))
        return fail(LABFM_EINVAL, "labfm_moment_systems: NULL array");
    Context* c = (Context*)ctx;
    DeviceGuard g(c->device);
    if (!g.ok) return fail(LABFM_EHIP, "labfm_moment_systems: hipSetDevice failed");
    WeightArgs a;
    one_set_args(a, x, y, n, dom, R, nullptr, row_ptr, col, nnz, opt, nullptr, nullptr, status, nullptr, nullptr);
    return moment_systems(c, a, k, M, psi, status, (hipStream_t)stream);
}

int64_t labfm_mlp_cache_floats(const labfm_mlp* net, int64_t B) {
    std::string why;
    if (!mlp_ok(net, why) || B < 0) return -1;
    return (int64_t)mlp_cache_floats(net, B);
}

labfm_err labfm_mlp_forward(void* ctx, const labfm_mlp* net, const float* in, int64_t B, float* out, float* cache,
                            int denorm, void* stream) {
    std::string why;
    if (!ctx) return fail(LABFM_EINVAL, "labfm_mlp_forward: ctx is NULL");
    if (!mlp_ok(net, why)) return fail(LABFM_EINVAL, "labfm_mlp_forward: " + why);
    if (B < 0 || B > INT32_MAX) return fail(LABFM_EINVAL, "labfm_mlp_forward: B out of range");
    if (B > 0 && (!in || !out)) return fail(LABFM_EINVAL, "labfm_mlp_forward: NULL array");
    if (denorm && (!net->mu || !net->sd)) return fail(LABFM_EINVAL, "labfm_mlp_forward: denorm needs mu and sd");
    Context* c = (Context*)ctx;
    DeviceGuard g(c->device);
    return mlp_forward(c, net, in, B, out, cache, denorm, (hipStream_t)stream);
}

labfm_err labfm_mlp_backward(void* ctx, const labfm_mlp* net, const float* in, const float* cache, const float* dout,
                             int64_t B, const labfm_mlp_grads* grads, void* stream) {
    std::string why;
    if (!ctx || !grads) return fail(LABFM_EINVAL, "labfm_mlp_backward: ctx or grads is NULL");
    if (!mlp_ok(net, why)) return fail(LABFM_EINVAL, "labfm_mlp_backward: " + why);
    if (B < 0 || B > INT32_MAX) return fail(LABFM_EINVAL, "labfm_mlp_backward: B out of range");
    if (B > 0 && (!in || !dout || (net->n_layers > 1 && !cache)))
        return fail(LABFM_EINVAL, "labfm_mlp_backward: NULL array");
    for (int l = 0; l < net->n_layers; ++l)
        if (!grads->W[l] || !grads->b[l]) return fail(LABFM_EINVAL, "labfm_mlp_backward: NULL gradient buffer");
    Context* c = (Context*)ctx;
    DeviceGuard g(c->device);
    return mlp_backward(c, net, in, cache, dout, B, grads, (hipStream_t)stream);
}

labfm_err labfm_mlp_moment_loss(void* ctx, const float* y, const float* M, const float* mu, const float* sd,
                                int order, unsigned ops, int64_t B, float* dy, double* loss, void* stream) {
    if (!ctx) return fail(LABFM_EINVAL, "labfm_mlp_moment_loss: ctx is NULL");
    if (order < 1 || order > LABFM_MAX_ORDER) return fail(LABFM_EINVAL, "labfm_mlp_moment_loss: order must be 1..8");
    if (ops == 0 || (ops & ~31u)) return fail(LABFM_EINVAL, "labfm_mlp_moment_loss: bad ops");
    if (B < 0) return fail(LABFM_EINVAL, "labfm_mlp_moment_loss: B < 0");
    if (B > 0 && (!y || !M || !mu || !sd || !dy || !loss)) return fail(LABFM_EINVAL, "labfm_mlp_moment_loss: NULL array");
    const int minord[5] = {1, 1, 2, 4, 6};
    for (int b = 0; b < 5; ++b)
        if (((ops >> b) & 1u) && order < minord[b])
            return fail(LABFM_EINVAL, "labfm_mlp_moment_loss: order too low for the operators");
    Context* c = (Context*)ctx;
    DeviceGuard g(c->device);
    return mlp_moment_loss(c, y, M, mu, sd, order, ops, B, dy, loss, (hipStream_t)stream);
}

labfm_err labfm_mlp_adam(void* ctx, float* param, const float* grad, float* m, float* v, void* param_bf16,
                         int64_t count, const labfm_adam* hp, int64_t t, void* stream) {
    if (!ctx || !hp) return fail(LABFM_EINVAL, "labfm_mlp_adam: ctx or hp is NULL");
    if (count < 0 || t < 1) return fail(LABFM_EINVAL, "labfm_mlp_adam: count < 0 or t < 1");
    if (count > 0 && (!param || !grad || !m || !v)) return fail(LABFM_EINVAL, "labfm_mlp_adam: NULL array");
    if (!(hp->beta1 >= 0.0 && hp->beta1 < 1.0 && hp->beta2 >= 0.0 && hp->beta2 < 1.0 && hp->eps > 0.0 &&
          std::isfinite(hp->lr)))
        return fail(LABFM_EINVAL, "labfm_mlp_adam: bad hyper-parameters");
    Context* c = (Context*)ctx;
    DeviceGuard g(c->device);
    return mlp_adam(c, param, grad, m, v, param_bf16, count, hp, t, (hipStream_t)stream);
}

labfm_err labfm_mlp_cast_bf16(void* ctx, const float* src, void* dst, int64_t count, void* stream) {
    if (!ctx) return fail(LABFM_EINVAL, "labfm_mlp_cast_bf16: ctx is NULL");
    if (count < 0) return fail(LABFM_EINVAL, "labfm_mlp_cast_bf16: count < 0");
    if (count > 0 && (!src || !dst)) return fail(LABFM_EINVAL, "labfm_mlp_cast_bf16: NULL array");
    Context* c = (Context*)ctx;
    DeviceGuard g(c->device);
    return mlp_cast_bf16(src, dst, count, (hipStream_t)stream);
}

labfm_err labfm_timing_enable(void* ctx, int enable) {
    if (!ctx) return fail(LABFM_EINVAL, "labfm_timing_enable: ctx is NULL");
    ((Context*)ctx)->timing = enable != 0;
    return LABFM_OK;
}

labfm_err labfm_timing_read(void* ctx, const char* filter, int64_t* launches, double* total_ms) {
    if (!ctx || !launches || !total_ms) return fail(LABFM_EINVAL, "labfm_timing_read: NULL argument");
    Context* c = (Context*)ctx;
    DeviceGuard g(c->device);
    *launches = 0;
    *total_ms = 0.0;
    std::vector<Context::Timed> keep;
    for (auto& t : c->timed) {
        bool match = !filter || t.name.find(filter) != std::string::npos;
        if (!match) {
            keep.push_back(t);
            continue;
        }
        LABFM_HIP_CHECK(hipEventSynchronize(t.b));
        float ms = 0.0f;
        LABFM_HIP_CHECK(hipEventElapsedTime(&ms, t.a, t.b));
        *total_ms += ms;
        *launches += 1;
        hipEventDestroy(t.a);
        hipEventDestroy(t.b);
    }
    c->timed.swap(keep);
    return LABFM_OK;
}

}  // extern "C"
