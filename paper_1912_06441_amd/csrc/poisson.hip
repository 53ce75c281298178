// poisson.hip -- global Laplacian solve (Sec. 5.2 of King, Lind & Nasar) on
// gfx950: A^L Phi = F, where row i of A^L applies the node's Laplacian weights
// in difference form (A_ij = w_ij, A_ii = -sum_j w_ij) and Dirichlet rows are
// identity rows.  Solver: BiCGStab with a Jacobi preconditioner applied on the
// right (van der Vorst 1992), FP64.
//
// Every scalar of the iteration (rho, alpha, omega, ...) lives in device
// memory and is produced by the kernel that finishes its reduction, so one
// iteration (two sparse products, three vector updates, three reductions;
// the residual update also forms (r, r) and the next (r0, r)) is captured
// once as a HIP graph and replayed without host round trips; the host reads the residual only every `check_every`
// iterations.  When the residual reaches the tolerance, or the recurrence
// breaks down, a flag in the same scalar block turns the remaining replays
// into no-ops, so the returned iterate is the one that met the test.
// Reductions use a fixed grid, so results do not depend on timing.
#include "labfm_internal.hpp"
#include "stencil_rows.hpp"

#include <algorithm>
#include <cmath>

namespace labfm {

namespace {

using namespace rows;

constexpr int DOT_BLOCKS = 512;
constexpr int DOT_THREADS = 256;

// scalar block
enum { S_RHO, S_RHO_OLD, S_ALPHA, S_OMEGA, S_BETA, S_RV, S_TS, S_TT, S_RR, S_BB, S_STOP, S_ITERS, S_TOL2, S_COUNT };
// S_STOP: 0 running, 1 converged, 2 breakdown

__device__ inline double block_sum(double v, double* sh) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    const int wid = threadIdx.x / 64, lane = threadIdx.x % 64;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x / 64); ++k) t += sh[k];
    __syncthreads();
    return t;  // valid in thread 0
}

// Sparse product rows: 8 lanes per row, 8 loads in flight per lane (measured
// best for one FP64 stream on 1024^2 order-6 rows: 0.36 ms per iteration
// against 0.41 ms at 16 x 4).
constexpr int SG = 8, SU = 8;

// y = A x (difference-form rows about center[i], or node i itself when center
// is NULL; identity rows where fixed[i] != 0)
__global__ __launch_bounds__(256) void k_spmv(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                              int64_t n, const double* __restrict__ w,
                                              const int8_t* __restrict__ fixed, const int32_t* __restrict__ center,
                                              const double* __restrict__ x, double* __restrict__ y,
                                              const double* __restrict__ S) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t row = gid / SG;
    const int sub = (int)(gid % SG);
    if (row >= n) return;  // whole groups exit together
    // the stop flag, the row bounds and the row's own values are requested
    // together, ahead of the dependent index and gather loads
    const bool stop = S && S[S_STOP] != 0.0;
    const int64_t s = rp[row], e = rp[row + 1];
    const double xr = x[row];
    const double xi = center ? x[center[row]] : xr;
    const bool ident = fixed && fixed[row];
    if (stop) return;
    WPtrs<double, 1> wp{{w}};
    double acc[1] = {0.0};
    row_sums<double, SG, SU, 1>(col, s, e, sub, wp, x, xi, acc);
    const double v = group_sum<double, SG>(acc[0]);
    if (sub == 0) y[row] = ident ? xr : v;
}

// inverse diagonal of A^L (1 on identity rows and where the diagonal is zero):
// the coefficient of x_i in row i, sum_{col[q] = i} w[q] - [center_i = i] sum_q w[q]
__global__ void k_jacobi(const int64_t* __restrict__ rp, const int32_t* __restrict__ col, int64_t n,
                         const double* __restrict__ w, const int8_t* __restrict__ fixed,
                         const int32_t* __restrict__ center, double* __restrict__ dinv) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool own = !center || center[i] == i;
    double d = 0.0;
    for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
        if (own) d -= w[q];
        if (col[q] == i) d += w[q];
    }
    if (fixed && fixed[i]) d = 1.0;
    dinv[i] = d != 0.0 ? 1.0 / d : 1.0;
}

// ---- rows of the enlarged system with Neumann ghost rows (Sec. 5.2, eq. neu)
__device__ inline int64_t nr_source(const int32_t* parent, int64_t i, int64_t n) {
    const int64_t p = parent ? (int64_t)parent[i] : -1;
    return (p >= 0 && p < n) ? p : i;  // an out-of-range parent counts as none
}
__global__ void k_nr_count(const int64_t* __restrict__ rp, const int32_t* __restrict__ parent, int64_t n,
                           int64_t* __restrict__ len) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t src = nr_source(parent, i, n);
    len[i] = rp[src + 1] - rp[src];
}
__global__ void k_nr_fill(const int64_t* __restrict__ rp, const int32_t* __restrict__ col, int64_t n,
                          const double* __restrict__ wx, const double* __restrict__ wy,
                          const double* __restrict__ wl, const int32_t* __restrict__ parent,
                          const double* __restrict__ nx, const double* __restrict__ ny,
                          const int64_t* __restrict__ orp, int32_t* __restrict__ ocol, double* __restrict__ ow,
                          int32_t* __restrict__ ocenter) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t src = nr_source(parent, i, n);
    const int64_t s = rp[src], e = rp[src + 1], o = orp[i];
    if (src == i) {
        for (int64_t q = s; q < e; ++q) {
            ocol[o + (q - s)] = col[q];
            ow[o + (q - s)] = wl[q];
        }
    } else {  // ghost row: the parent's normal derivative
        const double a = nx[i], b = ny[i];
        for (int64_t q = s; q < e; ++q) {
            ocol[o + (q - s)] = col[q];
            ow[o + (q - s)] = a * wx[q] + b * wy[q];
        }
    }
    ocenter[i] = (int32_t)src;
}

// partial sums of a.b and (optionally) c.d over a fixed grid of DOT_BLOCKS
__global__ __launch_bounds__(DOT_THREADS) void k_dot2(const double* __restrict__ a, const double* __restrict__ b,
                                                      const double* __restrict__ c, const double* __restrict__ d,
                                                      int64_t n, double* __restrict__ part,
                                                      const double* __restrict__ S) {
    __shared__ double sh[DOT_THREADS / 64];
    if (S && S[S_STOP] != 0.0) return;
    double s1 = 0.0, s2 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        s1 += a[i] * b[i];
        if (c) s2 += c[i] * d[i];
    }
    const double t1 = block_sum(s1, sh);
    const double t2 = block_sum(s2, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = t1;
        part[gridDim.x + blockIdx.x] = t2;
    }
}

enum { OP_BB, OP_RR0, OP_RV, OP_OMEGA, OP_RR_RHO };

constexpr int FINAL_THREADS = 512;

// sums nparts partials of each of the two sums (second array at part + nparts)
// and advances the scalar recurrence (one block, fixed summation order)
__global__ __launch_bounds__(FINAL_THREADS) void k_dot_final(const double* __restrict__ part, int nparts,
                                                             double* __restrict__ S, int op) {
    __shared__ double sh[FINAL_THREADS / 64];
    if (op != OP_BB && op != OP_RR0 && S[S_STOP] != 0.0) return;
    double s1 = 0.0, s2 = 0.0;
    for (int i = threadIdx.x; i < nparts; i += FINAL_THREADS) {
        s1 += part[i];
        s2 += part[nparts + i];
    }
    const double t1 = block_sum(s1, sh);
    const double t2 = block_sum(s2, sh);
    if (threadIdx.x != 0) return;
    switch (op) {
        case OP_BB:  // ||F||^2; initial scalars
            S[S_BB] = t1;
            S[S_RHO_OLD] = S[S_ALPHA] = S[S_OMEGA] = 1.0;
            S[S_ITERS] = 0.0;
            S[S_STOP] = 0.0;
            break;
        case OP_RR0:  // ||r0||^2 = (r0, r0): already converged?  First rho.
            S[S_RR] = t1;
            S[S_RHO] = t1;
            S[S_BETA] = 0.0;  // p = v = 0 at the start
            if (!(t1 > S[S_TOL2] * S[S_BB])) S[S_STOP] = 1.0;
            break;
        case OP_RV:
            S[S_RV] = t1;
            if (t1 == 0.0 || !std::isfinite(t1)) {
                S[S_STOP] = 2.0;
                break;
            }
            S[S_ALPHA] = S[S_RHO] / t1;
            break;
        case OP_OMEGA:
            S[S_TS] = t1;
            S[S_TT] = t2;
            S[S_OMEGA] = t2 > 0.0 ? t1 / t2 : 0.0;
            break;
        case OP_RR_RHO: {  // t1 = (r, r), t2 = (r0, r): test, then rho and beta of the next iteration
            S[S_RR] = t1;
            S[S_ITERS] += 1.0;
            if (!std::isfinite(t1)) {
                S[S_STOP] = 2.0;
                break;
            }
            if (t1 <= S[S_TOL2] * S[S_BB]) {
                S[S_STOP] = 1.0;
                break;
            }
            const double rho = t2;
            if (S[S_OMEGA] == 0.0 || rho == 0.0 || !std::isfinite(rho)) {
                S[S_STOP] = 2.0;
                break;
            }
            S[S_BETA] = (rho / S[S_RHO]) * (S[S_ALPHA] / S[S_OMEGA]);
            S[S_RHO_OLD] = S[S_RHO];
            S[S_RHO] = rho;
            break;
        }
    }
}

// r = F - t; r0 = r; p = v = 0
__global__ void k_init(int64_t n, const double* __restrict__ F, const double* __restrict__ t, double* __restrict__ r,
                       double* __restrict__ r0, double* __restrict__ p, double* __restrict__ v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double ri = F[i] - t[i];
    r[i] = ri;
    r0[i] = ri;
    p[i] = 0.0;
    v[i] = 0.0;
}

// p = r + beta (p - omega v); y = D^-1 p
__global__ void k_update_p(int64_t n, const double* __restrict__ S, const double* __restrict__ r,
                           const double* __restrict__ v, const double* __restrict__ dinv, double* __restrict__ p,
                           double* __restrict__ y) {
    if (S[S_STOP] != 0.0) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double pi = r[i] + S[S_BETA] * (p[i] - S[S_OMEGA] * v[i]);
    p[i] = pi;
    y[i] = dinv[i] * pi;
}

// x += alpha y; s = r - alpha v; y <- z = D^-1 s
__global__ void k_update_s(int64_t n, const double* __restrict__ S, const double* __restrict__ r,
                           const double* __restrict__ v, const double* __restrict__ dinv, double* __restrict__ x,
                           double* __restrict__ y, double* __restrict__ s) {
    if (S[S_STOP] != 0.0) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double a = S[S_ALPHA];
    x[i] += a * y[i];
    const double si = r[i] - a * v[i];
    s[i] = si;
    y[i] = dinv[i] * si;
}

// x += omega z; r = s - omega t; per-block partial sums of (r, r) and (r0, r)
__global__ __launch_bounds__(256) void k_update_r(int64_t n, const double* __restrict__ S,
                                                  const double* __restrict__ z, const double* __restrict__ s,
                                                  const double* __restrict__ t, const double* __restrict__ r0,
                                                  double* __restrict__ x, double* __restrict__ r,
                                                  double* __restrict__ part) {
    __shared__ double sh[4];
    if (S[S_STOP] != 0.0) return;  // uniform
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double rr = 0.0, r0r = 0.0;
    if (i < n) {
        const double om = S[S_OMEGA];
        x[i] += om * z[i];
        const double ri = s[i] - om * t[i];
        r[i] = ri;
        rr = ri * ri;
        r0r = r0[i] * ri;
    }
    const double p1 = block_sum(rr, sh);
    const double p2 = block_sum(r0r, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = p1;
        part[gridDim.x + blockIdx.x] = p2;
    }
}

struct Bufs {
    double *r, *r0, *p, *v, *y, *s, *t, *dinv, *part, *S;
};

inline unsigned spmv_blocks(int64_t n) { return (unsigned)((n * SG + 255) / 256); }

void enqueue_iteration(const labfm_poisson_plan* pl, double* x, const Bufs& b, hipStream_t st) {
    const int64_t n = pl->n;
    const unsigned nv = (unsigned)((n + 255) / 256);
    const unsigned nm = spmv_blocks(n);
    k_update_p<<<nv, 256, 0, st>>>(n, b.S, b.r, b.v, b.dinv, b.p, b.y);
    k_spmv<<<nm, 256, 0, st>>>(pl->row_ptr, pl->col, n, pl->w_lap, pl->fixed, pl->center, b.y, b.v, b.S);
    k_dot2<<<DOT_BLOCKS, DOT_THREADS, 0, st>>>(b.r0, b.v, nullptr, nullptr, n, b.part, b.S);
    k_dot_final<<<1, FINAL_THREADS, 0, st>>>(b.part, DOT_BLOCKS, b.S, OP_RV);
    k_update_s<<<nv, 256, 0, st>>>(n, b.S, b.r, b.v, b.dinv, x, b.y, b.s);
    k_spmv<<<nm, 256, 0, st>>>(pl->row_ptr, pl->col, n, pl->w_lap, pl->fixed, pl->center, b.y, b.t, b.S);
    k_dot2<<<DOT_BLOCKS, DOT_THREADS, 0, st>>>(b.t, b.s, b.t, b.t, n, b.part, b.S);
    k_dot_final<<<1, FINAL_THREADS, 0, st>>>(b.part, DOT_BLOCKS, b.S, OP_OMEGA);
    k_update_r<<<nv, 256, 0, st>>>(n, b.S, b.y, b.s, b.t, b.r0, x, b.r, b.part);
    k_dot_final<<<1, FINAL_THREADS, 0, st>>>(b.part, (int)nv, b.S, OP_RR_RHO);
}

__global__ void k_set_tol(double* S, double tol2) { S[S_TOL2] = tol2; }

}  // namespace

labfm_err poisson_solve(Context* c, const labfm_poisson_plan* pl, const double* F, double* x, double* scratch,
                        int* iters, double* rel_resid, int* converged, hipStream_t st) {
    const int64_t n = pl->n;
    const unsigned nv = (unsigned)((n + 255) / 256);
    const unsigned nm = spmv_blocks(n);
    const size_t nparts = std::max<size_t>((size_t)DOT_BLOCKS, (size_t)nv);
    labfm_err e = ensure(c->poisson, sizeof(double) * (2 * nparts + S_COUNT));
    if (e != LABFM_OK) return e;
    Bufs b{};
    b.r = scratch;
    b.r0 = scratch + n;
    b.p = scratch + 2 * n;
    b.v = scratch + 3 * n;
    b.y = scratch + 4 * n;
    b.s = scratch + 5 * n;
    b.t = scratch + 6 * n;
    b.dinv = scratch + 7 * n;
    b.part = (double*)c->poisson.p;
    b.S = b.part + 2 * nparts;
    {
        KernelTimer timer(c, "poisson_setup", st);
        k_set_tol<<<1, 1, 0, st>>>(b.S, pl->tol * pl->tol);
        k_dot2<<<DOT_BLOCKS, DOT_THREADS, 0, st>>>(F, F, nullptr, nullptr, n, b.part, nullptr);
        k_dot_final<<<1, FINAL_THREADS, 0, st>>>(b.part, DOT_BLOCKS, b.S, OP_BB);
        k_jacobi<<<nv, 256, 0, st>>>(pl->row_ptr, pl->col, n, pl->w_lap, pl->fixed, pl->center, b.dinv);
        k_spmv<<<nm, 256, 0, st>>>(pl->row_ptr, pl->col, n, pl->w_lap, pl->fixed, pl->center, x, b.t, nullptr);
        k_init<<<nv, 256, 0, st>>>(n, F, b.t, b.r, b.r0, b.p, b.v);
        k_dot2<<<DOT_BLOCKS, DOT_THREADS, 0, st>>>(b.r, b.r, nullptr, nullptr, n, b.part, nullptr);
        k_dot_final<<<1, FINAL_THREADS, 0, st>>>(b.part, DOT_BLOCKS, b.S, OP_RR0);
        LABFM_HIP_CHECK(hipGetLastError());
    }
    // one iteration as a graph, captured on a private stream
    hipStream_t cap;
    LABFM_HIP_CHECK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        hipStreamDestroy(cap);
        set_error("labfm_poisson_solve: hipStreamBeginCapture failed");
        return LABFM_EHIP;
    }
    enqueue_iteration(pl, x, b, cap);
    hipError_t he = hipStreamEndCapture(cap, &graph);
    hipGraphExec_t exec = nullptr;
    if (he == hipSuccess) he = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) hipGraphDestroy(graph);
    hipStreamDestroy(cap);
    if (he != hipSuccess) {
        set_error(std::string("labfm_poisson_solve: graph capture: ") + hipGetErrorString(he));
        return LABFM_EHIP;
    }
    double hs[S_COUNT];
    int done = 0;
    labfm_err out = LABFM_OK;
    {
        KernelTimer timer(c, "poisson_iterations", st);
        for (;;) {
            if (hipMemcpyAsync(hs, b.S, sizeof(hs), hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess) {
                set_error("labfm_poisson_solve: reading the residual failed");
                out = LABFM_EHIP;
                break;
            }
            if (hs[S_STOP] != 0.0 || done >= pl->max_iters) break;
            const int k = std::min(pl->check_every, pl->max_iters - done);
            for (int q = 0; q < k; ++q)
                if (hipGraphLaunch(exec, st) != hipSuccess) {
                    set_error("labfm_poisson_solve: hipGraphLaunch failed");
                    out = LABFM_EHIP;
                    break;
                }
            if (out != LABFM_OK) break;
            done += k;
        }
    }
    hipGraphExecDestroy(exec);
    if (out != LABFM_OK) return out;
    if (iters) *iters = (int)hs[S_ITERS];
    if (rel_resid) *rel_resid = hs[S_BB] > 0.0 ? std::sqrt(hs[S_RR] / hs[S_BB]) : 0.0;
    if (converged) *converged = hs[S_STOP] == 1.0 ? 1 : 0;
    return LABFM_OK;
}

labfm_err neumann_rows(Context* c, const int64_t* rp, const int32_t* col, int64_t n, const double* wx,
                       const double* wy, const double* wl, const int32_t* parent, const double* nx, const double* ny,
                       int64_t* orp, int32_t* ocol, double* ow, int32_t* ocenter, int64_t* nnz_host, hipStream_t st) {
    const unsigned nb = (unsigned)((n + 255) / 256);
    if (!ocol) {  // count pass
        labfm_err e = ensure(c->counts, sizeof(int64_t) * (size_t)n);
        if (e != LABFM_OK) return e;
        int64_t* len = (int64_t*)c->counts.p;
        k_nr_count<<<nb, 256, 0, st>>>(rp, parent, n, len);
        LABFM_HIP_CHECK(hipGetLastError());
        if ((e = exclusive_scan_i64(c, len, orp, n, st)) != LABFM_OK) return e;
        LABFM_HIP_CHECK(hipMemcpyAsync(nnz_host, orp + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        LABFM_HIP_CHECK(hipStreamSynchronize(st));
        return LABFM_OK;
    }
    k_nr_fill<<<nb, 256, 0, st>>>(rp, col, n, wx, wy, wl, parent, nx, ny, orp, ocol, ow, ocenter);
    LABFM_HIP_CHECK(hipGetLastError());
    return LABFM_OK;
}

}  // namespace labfm
