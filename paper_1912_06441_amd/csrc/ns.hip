// ns.hip -- incompressible Navier-Stokes in vorticity-streamfunction form
// (Sec. 5.4 of King, Lind & Nasar) on gfx950:
//   d omega/dt = -(u L^x(omega) + v L^y(omega)) + nu L^L(omega),
//   L^L psi = -omega (global solve, Sec. 5.2),  u = L^y(psi),  v = -L^x(psi),
// classical RK4; at every stage the stream function is re-solved (BiCGStab,
// warm-started from the previous stage's psi) and the velocity taken from its
// stencil derivatives.  Per stage: one source kernel, the Krylov solve, one
// velocity pass (two weight streams over psi) and one vorticity pass (three
// weight streams over omega and the stage update).
#include "labfm_internal.hpp"
#include "stencil_rows.hpp"

namespace labfm {

namespace {

using namespace rows;

// F = -omega, 0 on the pinned (Dirichlet) rows of the stream-function solve
__global__ void k_ns_source(int64_t n, const double* __restrict__ om, const int8_t* __restrict__ fixed,
                            double* __restrict__ F) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    F[i] = (fixed && fixed[i]) ? 0.0 : -om[i];
}

// u = L^y(psi), v = -L^x(psi), one read of the index stream
__global__ __launch_bounds__(256) void k_ns_velocity(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                     int64_t n, const double* __restrict__ wx,
                                                     const double* __restrict__ wy, const double* __restrict__ psi,
                                                     double* __restrict__ u, double* __restrict__ v) {
    constexpr int G = Shape<double>::G, U = Shape<double>::U;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t row = gid / G;
    const int sub = (int)(gid % G);
    if (row >= n) return;
    WPtrs<double, 2> wp{{wy, wx}};
    double a[2] = {0.0, 0.0};
    row_sums<double, G, U, 2>(col, rp[row], rp[row + 1], sub, wp, psi, psi[row], a);
    const double dy = group_sum<double, G>(a[0]);
    const double dx = group_sum<double, G>(a[1]);
    if (sub == 0) {
        u[row] = dy;
        v[row] = -dx;
    }
}

// k = -(u L^x(om) + v L^y(om)) + nu L^L(om) at the stage state, then the RK4 stage update
__global__ __launch_bounds__(256) void k_ns_stage(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                  int64_t n, WPtrs<double, 3> w, const double* om_in,
                                                  const double* __restrict__ u, const double* __restrict__ v,
                                                  double nu, double dt, int stage, double* om, double* acc,
                                                  double* om_out) {
    constexpr int G = Shape<double>::G, U = Shape<double>::U;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t row = gid / G;
    const int sub = (int)(gid % G);
    if (row >= n) return;
    const Rk4Node<double> node = rk4_load<double>(stage, row, nullptr, om, acc);
    const double ui = u[row], vi = v[row];
    double a[3] = {0.0, 0.0, 0.0};
    row_sums<double, G, U, 3>(col, rp[row], rp[row + 1], sub, w, om_in, om_in[row], a);
#pragma unroll
    for (int d = 0; d < 3; ++d) a[d] = group_sum<double, G>(a[d]);
    if (sub != 0) return;
    const double k = -(ui * a[0] + vi * a[1]) + nu * a[2];
    rk4_store<double>(stage, k, dt, row, node, om, acc, om_out);
}

}  // namespace

labfm_err ns_step(Context* c, const labfm_ns_plan* p, double* om, double* psi, double* scratch, int nsteps,
                  int* solver_iters, int* all_converged, hipStream_t st) {
    const int64_t n = p->n;
    double* F = scratch;
    double* u = scratch + n;
    double* v = scratch + 2 * n;
    double* omA = scratch + 3 * n;
    double* omB = scratch + 4 * n;
    double* acc = scratch + 5 * n;
    double* kry = scratch + 6 * n;  // 8 n for the Krylov solve
    const double* in[4] = {om, omA, omB, omA};
    double* outs[4] = {omA, omB, omA, om};
    labfm_poisson_plan pp{};
    pp.row_ptr = p->row_ptr;
    pp.col = p->col;
    pp.n = n;
    pp.nnz = p->nnz;
    pp.w_lap = p->w_lap;
    pp.fixed = p->psi_fixed;
    pp.tol = p->tol;
    pp.max_iters = p->max_iters;
    pp.check_every = p->check_every;
    WPtrs<double, 3> w{{p->w_x, p->w_y, p->w_lap}};
    const unsigned nv = (unsigned)((n + 255) / 256);
    const unsigned nm = blocks_for<double>(n);
    long long total = 0;
    int ok_all = 1;
    for (int s = 0; s < nsteps; ++s)
        for (int stage = 0; stage < 4; ++stage) {
            k_ns_source<<<nv, 256, 0, st>>>(n, in[stage], p->psi_fixed, F);
            LABFM_HIP_CHECK(hipGetLastError());
            int it = 0, conv = 0;
            double res = 0.0;
            labfm_err e = poisson_solve(c, &pp, F, psi, kry, &it, &res, &conv, st);
            if (e != LABFM_OK) return e;
            total += it;
            if (!conv) ok_all = 0;
            KernelTimer timer(c, "ns_stage", st);
            k_ns_velocity<<<nm, 256, 0, st>>>(p->row_ptr, p->col, n, p->w_x, p->w_y, psi, u, v);
            k_ns_stage<<<nm, 256, 0, st>>>(p->row_ptr, p->col, n, w, in[stage], u, v, p->nu, p->dt, stage, om, acc,
                                           outs[stage]);
            LABFM_HIP_CHECK(hipGetLastError());
        }
    if (solver_iters) *solver_iters = (int)(total > 2147483647LL ? 2147483647LL : total);
    if (all_converged) *all_converged = ok_all;
    return LABFM_OK;
}

}  // namespace labfm
