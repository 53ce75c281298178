// weights.hip -- per-node LABFM weights on gfx950, FP64 path.
//
// For node i of order k (Sec. 3.1 of King, Lind & Nasar): h = R_i / 2,
// d_j = r_ji / h, M = sum_j X(d_j) W(d_j)^T (eq. disc_form), M Psi^d = C^d
// (eq. lsys), w^d_j = W(d_j) . Psi^d (eq. w_abf), then w^d /= h^l(d).  The
// paper names no solver; here M is equilibrated (rows, then columns, by their
// max-abs entry), LU-factorised with partial pivoting, and the weights are
// refined in FP64 on the moment residual r = C - X^T w (w += W M^-1 r).
//
// Launch shape: one 64-lane wavefront (one workgroup) per node system, a
// persistent grid striding over a per-order work list.  M lives in LDS;
// basis values are produced in LDS chunks and M is accumulated in registers
// (each lane owns a BS x BS block of the padded 8BS x 8BS matrix).
#include "weights_common.hpp"

namespace labfm {

namespace {
using namespace wk;

template <int K, int FAM>
__global__ __launch_bounds__(64) void k_weights_fp64(WeightArgs a, OpList ops, const int32_t* list,
                                                     const int32_t* list_off, const int32_t* list_cnt) {
    constexpr int P = p_of_k(K);
    constexpr int BS = (P + 7) / 8;
    constexpr int PP = 8 * BS;
    constexpr int LD = P + 1;
    constexpr int JS = NMAX / 64;  // neighbour slots per lane

    __shared__ double sM[P * LD];
    __shared__ double sChunk[2 * CH * PP];  // basis chunk: X then W
    __shared__ double sD[2][NMAX];          // scaled offsets
    __shared__ double sWl[MAXOPS][NMAX];    // scaled weights (for the residual)
    __shared__ double sPsi[MAXOPS][PP];     // solution / correction coefficients
    __shared__ double sRs[P], sCs[P];
    __shared__ int sPerm[P];

    const int lane = threadIdx.x;
    const int nops = ops.nops;
    const int count = list_cnt[K];
    const int32_t* mylist = list + list_off[K];

    for (int t = blockIdx.x; t < count; t += gridDim.x) {
        NodeSet S;
        int64_t i;
        resolve(a, mylist[t], S, i);
        const int64_t s0 = S.row_ptr[i];
        const int N = (int)(S.row_ptr[i + 1] - s0);
        const double h = 0.5 * S.R[i];
        int status = LABFM_ST_OK;
        double res = INFINITY;
        int iters = 0;

        // block-uniform early exits
        for (int d = 0; d < nops; ++d)
            if (K < min_order(ops.op[d])) status = LABFM_ST_ORDER_TOO_LOW;
        if (status == LABFM_ST_OK && N < P) status = LABFM_ST_TOO_FEW;
        if (status == LABFM_ST_OK && N > NMAX) status = LABFM_ST_TOO_MANY;

        double dxr[JS], dyr[JS];
        if (status == LABFM_ST_OK) {
            const double xi = S.x[i], yi = S.y[i];
            bool bad = false;
#pragma unroll
            for (int js = 0; js < JS; ++js) {
                int q = lane + 64 * js;
                dxr[js] = 0.0;
                dyr[js] = 0.0;
                if (q < N) {
                    int32_t j = S.col[s0 + q];
                    dxr[js] = min_image(S.x[j] - xi, S.Lx, S.perx) / h;
                    dyr[js] = min_image(S.y[j] - yi, S.Ly, S.pery) / h;
                    sD[0][q] = dxr[js];
                    sD[1][q] = dyr[js];
                    if (FAM != LABFM_ABF_HERMITE && dxr[js] == 0.0 && dyr[js] == 0.0) bad = true;
                }
            }
            if (__any(bad)) status = LABFM_ST_DEGENERATE;
        }
        __syncthreads();

        if (status == LABFM_ST_OK) {
            // ---- assembly: M = sum_j X(d_j) W(d_j)^T, register-blocked
            const int lr = lane / 8, lc = lane % 8;
            double acc[BS][BS];
#pragma unroll
            for (int r = 0; r < BS; ++r)
#pragma unroll
                for (int c = 0; c < BS; ++c) acc[r][c] = 0.0;
            double* sX = sChunk;
            double* sW = sChunk + CH * PP;
            for (int j0 = 0; j0 < N; j0 += CH) {
                if (lane < 2 * CH) {
                    const int jj = lane % CH;
                    const int j = j0 + jj;
                    double* dst = (lane < CH ? sX : sW) + jj * PP;
                    if (j < N) {
                        BasisState<K> B;
                        basis_prepare<K, FAM>(B, sD[0][j], sD[1][j], a.rbf, a.sigma);
                        if (lane < CH) {
#pragma unroll
                            for (int m = 0; m < P; ++m) dst[m] = monomial<K>(B, m);
                        } else {
#pragma unroll
                            for (int m = 0; m < P; ++m) dst[m] = abf<K, FAM>(B, m);
                        }
                    } else {
#pragma unroll
                        for (int m = 0; m < P; ++m) dst[m] = 0.0;
                    }
#pragma unroll
                    for (int m = P; m < PP; ++m) dst[m] = 0.0;
                }
                __syncthreads();
                const int jmax = min(CH, N - j0);
                for (int jj = 0; jj < jmax; ++jj) {
                    double xv[BS], wv[BS];
#pragma unroll
                    for (int r = 0; r < BS; ++r) xv[r] = sX[jj * PP + lr * BS + r];
#pragma unroll
                    for (int c = 0; c < BS; ++c) wv[c] = sW[jj * PP + lc * BS + c];
#pragma unroll
                    for (int r = 0; r < BS; ++r)
#pragma unroll
                        for (int c = 0; c < BS; ++c) acc[r][c] = fma(xv[r], wv[c], acc[r][c]);
                }
                __syncthreads();
            }
#pragma unroll
            for (int r = 0; r < BS; ++r)
#pragma unroll
                for (int c = 0; c < BS; ++c) {
                    int m = lr * BS + r, nn = lc * BS + c;
                    if (m < P && nn < P) sM[m * LD + nn] = acc[r][c];
                }
            __syncthreads();

            // ---- equilibration: rows, then columns
            bool sing = false;
            if (lane < P) {
                double mx = 0.0;
                for (int c = 0; c < P; ++c) mx = fmax(mx, fabs(sM[lane * LD + c]));
                if (!(mx > 0.0) || !isfinite(mx)) sing = true;
                double rs = 1.0 / mx;
                sRs[lane] = rs;
                for (int c = 0; c < P; ++c) sM[lane * LD + c] *= rs;
            }
            __syncthreads();
            if (lane < P) {
                double mx = 0.0;
                for (int r = 0; r < P; ++r) mx = fmax(mx, fabs(sM[r * LD + lane]));
                if (!(mx > 0.0) || !isfinite(mx)) sing = true;
                double cs = 1.0 / mx;
                sCs[lane] = cs;
                for (int r = 0; r < P; ++r) sM[r * LD + lane] *= cs;
            }
            __syncthreads();
            if (__any(sing)) status = LABFM_ST_SINGULAR;

            // ---- LU with partial pivoting (ties: lowest row)
            int perm = lane;
            if (status == LABFM_ST_OK) {
                for (int kk = 0; kk < P; ++kk) {
                    // pivot: largest |M[r][kk]| over r >= kk, ties to the lowest row
                    const double v = (lane >= kk && lane < P) ? fabs(sM[lane * LD + kk]) : -1.0;
                    const double vmax = wave_max_double(v);
                    const unsigned long long hit = __ballot(v == vmax);
                    if (!(vmax > 0.0) || !isfinite(vmax) || hit == 0ull) {
                        status = LABFM_ST_SINGULAR;
                        break;
                    }
                    const int pr = __ffsll((long long)hit) - 1;
                    if (pr != kk) {
                        if (lane < P) {
                            const double u = sM[kk * LD + lane];
                            sM[kk * LD + lane] = sM[pr * LD + lane];
                            sM[pr * LD + lane] = u;
                        }
                        // permutation bookkeeping: position kk <-> pr
                        const int pk = __builtin_amdgcn_readlane(perm, kk), pp = __builtin_amdgcn_readlane(perm, pr);
                        if (lane == kk) perm = pp;
                        if (lane == pr) perm = pk;
                    }
                    __syncthreads();
                    // one pass: lane c > kk updates column c of the trailing rows, lane kk
                    // stores the multipliers l_r = M[r][kk] / M[kk][kk] (every lane reads
                    // M[r][kk] before lane kk overwrites it; rows in groups of eight)
                    if (lane >= kk && lane < P) {
                        const double inv = 1.0 / sM[kk * LD + kk];
                        const double u = sM[kk * LD + lane];
                        const bool own = lane == kk;
                        int r = kk + 1;
                        for (; r + 8 <= P; r += 8) {
                            double l[8], a[8];
#pragma unroll
                            for (int e = 0; e < 8; ++e) {
                                l[e] = sM[(r + e) * LD + kk];
                                a[e] = sM[(r + e) * LD + lane];
                            }
#pragma unroll
                            for (int e = 0; e < 8; ++e) {
                                const double m = l[e] * inv;
                                sM[(r + e) * LD + lane] = own ? m : fma(-m, u, a[e]);
                            }
                        }
                        for (; r < P; ++r) {
                            const double m = sM[r * LD + kk] * inv;
                            const double a0 = sM[r * LD + lane];
                            sM[r * LD + lane] = own ? m : fma(-m, u, a0);
                        }
                    }
                    __syncthreads();
                }
            }
            if (lane < P) sPerm[lane] = perm;
            __syncthreads();

            if (status == LABFM_ST_OK) {
                // ---- initial solve: lane m holds C^d[m]
                double b[MAXOPS];
#pragma unroll
                for (int d = 0; d < MAXOPS; ++d) b[d] = (d < nops) ? target(ops.op[d], lane) : 0.0;
                lu_solve<P, LD>(sM, sRs, sCs, sPerm, b, nops);
                if (lane < P)
#pragma unroll
                    for (int d = 0; d < MAXOPS; ++d)
                        if (d < nops) sPsi[d][lane] = b[d];
                __syncthreads();

                // ---- w_j = W(d_j) . Psi
                double wreg[JS][MAXOPS];
#pragma unroll
                for (int js = 0; js < JS; ++js) {
                    int q = lane + 64 * js;
#pragma unroll
                    for (int d = 0; d < MAXOPS; ++d) wreg[js][d] = 0.0;
                    if (q < N) {
                        BasisState<K> B;
                        basis_prepare<K, FAM>(B, dxr[js], dyr[js], a.rbf, a.sigma);
#pragma unroll
                        for (int m = 0; m < P; ++m) {
                            double wm = abf<K, FAM>(B, m);
#pragma unroll
                            for (int d = 0; d < MAXOPS; ++d)
                                if (d < nops) wreg[js][d] = fma(wm, sPsi[d][m], wreg[js][d]);
                        }
#pragma unroll
                        for (int d = 0; d < MAXOPS; ++d)
                            if (d < nops) sWl[d][q] = wreg[js][d];
                    }
                }
                __syncthreads();

                // ---- refinement on the moment residual (FP64)
                const int ma = lane < P ? ELEM.a[lane] : 0;
                const int mb = lane < P ? ELEM.b[lane] : 0;
                const double mf = lane < P ? inv_fact(ma) * inv_fact(mb) : 0.0;
                for (;;) {
                    double r[MAXOPS];
#pragma unroll
                    for (int d = 0; d < MAXOPS; ++d) r[d] = 0.0;
                    if (lane < P) {
                        double accr[MAXOPS];
#pragma unroll
                        for (int d = 0; d < MAXOPS; ++d) accr[d] = 0.0;
                        for (int q = 0; q < N; ++q) {
                            const double dx = sD[0][q], dy = sD[1][q];
                            double xm = mf;
#pragma unroll
                            for (int e = 0; e < K; ++e) {
                                xm *= (e < ma) ? dx : 1.0;
                                xm *= (e < mb) ? dy : 1.0;
                            }
#pragma unroll
                            for (int d = 0; d < MAXOPS; ++d)
                                if (d < nops) accr[d] = fma(xm, sWl[d][q], accr[d]);
                        }
#pragma unroll
                        for (int d = 0; d < MAXOPS; ++d)
                            if (d < nops) r[d] = target(ops.op[d], lane) - accr[d];
                    }
                    double rm = 0.0;
#pragma unroll
                    for (int d = 0; d < MAXOPS; ++d) {
                        const double ar = fabs(r[d]);
                        rm = (ar > rm || ar != ar) ? ar : rm;  // NaN propagates (fmax would drop it)
                    }
                    if (!isfinite(rm)) rm = INFINITY;
                    res = wave_max(rm);
                    if (!(res > a.tol_stop) || iters >= a.max_iters) break;
                    lu_solve<P, LD>(sM, sRs, sCs, sPerm, r, nops);
                    __syncthreads();
                    if (lane < P)
#pragma unroll
                        for (int d = 0; d < MAXOPS; ++d)
                            if (d < nops) sPsi[d][lane] = r[d];
                    __syncthreads();
#pragma unroll
                    for (int js = 0; js < JS; ++js) {
                        int q = lane + 64 * js;
                        if (q < N) {
                            BasisState<K> B;
                            basis_prepare<K, FAM>(B, dxr[js], dyr[js], a.rbf, a.sigma);
                            double dw[MAXOPS];
#pragma unroll
                            for (int d = 0; d < MAXOPS; ++d) dw[d] = 0.0;
#pragma unroll
                            for (int m = 0; m < P; ++m) {
                                double wm = abf<K, FAM>(B, m);
#pragma unroll
                                for (int d = 0; d < MAXOPS; ++d)
                                    if (d < nops) dw[d] = fma(wm, sPsi[d][m], dw[d]);
                            }
#pragma unroll
                            for (int d = 0; d < MAXOPS; ++d)
                                if (d < nops) {
                                    wreg[js][d] += dw[d];
                                    sWl[d][q] = wreg[js][d];
                                }
                        }
                    }
                    __syncthreads();
                    ++iters;
                }
                if (!(res <= a.tol_pass)) status = LABFM_ST_NOT_CONVERGED;

                // ---- unscale and store
#pragma unroll
                for (int d = 0; d < MAXOPS; ++d) {
                    if (d >= nops) continue;
                    double hl = 1.0;
                    for (int e = 0; e < deriv_order(ops.op[d]); ++e) hl *= h;
#pragma unroll
                    for (int js = 0; js < JS; ++js) {
                        int q = lane + 64 * js;
                        if (q < N) {
                            double wv = wreg[js][d] / hl;
                            if (S.w64) S.w64[(int64_t)d * S.nnz + s0 + q] = wv;
                            if (S.w32) S.w32[(int64_t)d * S.nnz + s0 + q] = (float)wv;
                        }
                    }
                }
            }
        }
        const bool failed = !(status == LABFM_ST_OK || status == LABFM_ST_NOT_CONVERGED);
        if (failed) {
            for (int d = 0; d < nops; ++d)
                for (int q = lane; q < N; q += 64) {
                    if (S.w64) S.w64[(int64_t)d * S.nnz + s0 + q] = 0.0;
                    if (S.w32) S.w32[(int64_t)d * S.nnz + s0 + q] = 0.0f;
                }
            res = INFINITY;
            iters = 0;
        }
        if (lane == 0) {
            S.status[i] = (int8_t)status;
            if (S.resid) S.resid[i] = (float)res;
            if (S.iters) S.iters[i] = (int8_t)(iters + a.iters_offset);
        }
        __syncthreads();
    }
}

// ---- per-order work lists: counting sort of node indices by order, with a
// workgroup-level histogram in LDS so that each workgroup issues one global
// atomic per order class.
__global__ __launch_bounds__(256) void k_list_count(const int8_t* order, int64_t n, int32_t* cnt /* [KMAX+2] */) {
    __shared__ int32_t h[KMAX + 1];
    if (threadIdx.x <= KMAX) h[threadIdx.x] = 0;
    __syncthreads();
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        int k = order[i];
        if (k < 1 || k > KMAX) k = 0;
        atomicAdd(&h[k], 1);
    }
    __syncthreads();
    if (threadIdx.x <= KMAX && h[threadIdx.x]) atomicAdd(&cnt[threadIdx.x], h[threadIdx.x]);
}
__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_list_offsets(const int32_t* cnt, int32_t* off) {
    if (threadIdx.x == 0) {
        int32_t run = 0;
        for (int k = 0; k <= KMAX; ++k) {
            off[k] = run;
            run += cnt[k];
        }
    }
}
__global__ __launch_bounds__(256) void k_list_scatter(const int8_t* order, int64_t n, int64_t base_g,
                                                      const int32_t* off, int32_t* fill, int32_t* list) {
    __shared__ int32_t h[KMAX + 1], base[KMAX + 1];
    if (threadIdx.x <= KMAX) h[threadIdx.x] = 0;
    __syncthreads();
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int k = 0, pos = 0;
    if (i < n) {
        k = order[i];
        if (k < 1 || k > KMAX) k = 0;
        pos = atomicAdd(&h[k], 1);
    }
    __syncthreads();
    if (threadIdx.x <= KMAX) base[threadIdx.x] = h[threadIdx.x] ? atomicAdd(&fill[threadIdx.x], h[threadIdx.x]) : 0;
    __syncthreads();
    if (i < n) list[off[k] + base[k] + pos] = (int32_t)(base_g + i);
}
// nodes with an invalid order: zero weights and status
__global__ void k_invalid_order(WeightArgs a, int nops, const int32_t* list, const int32_t* off, const int32_t* cnt) {
    int c = cnt[0];
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < c; t += gridDim.x * blockDim.x) {
        NodeSet S;
        int64_t i;
        resolve(a, list[off[0] + t], S, i);
        int64_t s0 = S.row_ptr[i], e0 = S.row_ptr[i + 1];
        for (int d = 0; d < nops; ++d)
            for (int64_t q = s0; q < e0; ++q) {
                if (S.w64) S.w64[(int64_t)d * S.nnz + q] = 0.0;
                if (S.w32) S.w32[(int64_t)d * S.nnz + q] = 0.0f;
            }
        S.status[i] = LABFM_ST_ORDER_TOO_LOW;
        if (S.resid) S.resid[i] = INFINITY;
        if (S.iters) S.iters[i] = 0;
    }
}

template <int K, int FAM>
int grid_for() {
    static int g = 0;
    if (g == 0) {
        int dev = 0, ncu = 0, per = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_weights_fp64<K, FAM>, 64, 0);
        if (ncu <= 0) ncu = 256;
        if (per <= 0) per = 1;
        g = ncu * per;
    }
    return g;
}

template <int FAM>
void launch_grids_all() {
    (void)grid_for<1, FAM>();
    (void)grid_for<2, FAM>();
    (void)grid_for<3, FAM>();
    (void)grid_for<4, FAM>();
    (void)grid_for<5, FAM>();
    (void)grid_for<6, FAM>();
    (void)grid_for<7, FAM>();
    (void)grid_for<8, FAM>();
}

template <int K, int FAM>
void launch_one(Context* c, const WeightArgs& a, const OpList& ops, const int32_t* list, const int32_t* off,
                const int32_t* cnt, unsigned mask, hipStream_t st) {
    if (!((mask >> K) & 1u)) return;
    static const char* names[KMAX + 1] = {"", "weights64_k1", "weights64_k2", "weights64_k3", "weights64_k4",
                                          "weights64_k5", "weights64_k6", "weights64_k7", "weights64_k8"};
    KernelTimer timer(c, names[K], st);
    k_weights_fp64<K, FAM><<<grid_for<K, FAM>(), 64, 0, st>>>(a, ops, list, off, cnt);
}

template <int FAM>
void launch_all(Context* c, const WeightArgs& a, const OpList& ops, const int32_t* list, const int32_t* off,
                const int32_t* cnt, unsigned mask, hipStream_t st) {
    launch_one<1, FAM>(c, a, ops, list, off, cnt, mask, st);
    launch_one<2, FAM>(c, a, ops, list, off, cnt, mask, st);
    launch_one<3, FAM>(c, a, ops, list, off, cnt, mask, st);
    launch_one<4, FAM>(c, a, ops, list, off, cnt, mask, st);
    launch_one<5, FAM>(c, a, ops, list, off, cnt, mask, st);
    launch_one<6, FAM>(c, a, ops, list, off, cnt, mask, st);
    launch_one<7, FAM>(c, a, ops, list, off, cnt, mask, st);
    launch_one<8, FAM>(c, a, ops, list, off, cnt, mask, st);
}

}  // namespace

// Grid sizes are found on first use (occupancy queries); done up front here so
// that no query happens while a stream is being captured.
void init_weight_grids() {
    launch_grids_all<LABFM_ABF_HERMITE>();
    launch_grids_all<LABFM_ABF_PAPER>();
    launch_grids_all<LABFM_ABF_PAPER_D1>();
}

labfm_err fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st) {
    if (n <= 0) return LABFM_OK;
    k_fill_i32<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(p, n, v);
    LABFM_HIP_CHECK(hipGetLastError());
    return LABFM_OK;
}

// Per-order work lists of global indices over every node set.  wl: at least
// ntotal + 3 (KMAX + 2) int32.  Counters are cleared with a kernel (no memset
// node when captured).
labfm_err build_order_lists(Context* c, const WeightArgs& a, const NodeSet* hs, hipStream_t st, int32_t** list,
                            int32_t** off, int32_t** cnt) {
    (void)c;
    int32_t* base = *list;  // caller's buffer on entry
    *cnt = base;
    int32_t* fill = base + (KMAX + 2);
    *off = base + 2 * (KMAX + 2);
    *list = base + 3 * (KMAX + 2);
    labfm_err e = fill_i32(base, 3 * (KMAX + 2), 0, st);
    if (e != LABFM_OK) return e;
    const int ns = a.nsets <= 1 ? 1 : a.nsets;
    for (int s = 0; s < ns; ++s) {
        if (hs[s].n <= 0) continue;
        k_list_count<<<(unsigned)((hs[s].n + 255) / 256), 256, 0, st>>>(hs[s].order, hs[s].n, *cnt);
    }
    k_list_offsets<<<1, 1, 0, st>>>(*cnt, *off);
    int64_t g0 = 0;
    for (int s = 0; s < ns; ++s) {
        if (hs[s].n > 0)
            k_list_scatter<<<(unsigned)((hs[s].n + 255) / 256), 256, 0, st>>>(hs[s].order, hs[s].n, g0, *off, fill,
                                                                             *list);
        g0 += hs[s].n;
    }
    LABFM_HIP_CHECK(hipGetLastError());
    return LABFM_OK;
}

labfm_err weights_fp64_lists(Context* c, const WeightArgs& a, const int32_t* list, const int32_t* off,
                             const int32_t* cnt, unsigned mask, hipStream_t st) {
    OpList ops{};  // unused slots stay 0: a zero target
    ops.nops = 0;
    for (int b = 0; b < 5; ++b)
        if (a.ops & (1u << b)) ops.op[ops.nops++] = 1u << b;
    if (a.abf == LABFM_ABF_HERMITE)
        launch_all<LABFM_ABF_HERMITE>(c, a, ops, list, off, cnt, mask, st);
    else if (a.abf == LABFM_ABF_PAPER)
        launch_all<LABFM_ABF_PAPER>(c, a, ops, list, off, cnt, mask, st);
    else
        launch_all<LABFM_ABF_PAPER_D1>(c, a, ops, list, off, cnt, mask, st);
    LABFM_HIP_CHECK(hipGetLastError());
    return LABFM_OK;
}

labfm_err weights_invalid_orders(const WeightArgs& a, const int32_t* list, const int32_t* off, const int32_t* cnt,
                                 hipStream_t st) {
    int nops = 0;
    for (int b = 0; b < 5; ++b) nops += (a.ops >> b) & 1u;
    k_invalid_order<<<64, 256, 0, st>>>(a, nops, list, off, cnt);
    LABFM_HIP_CHECK(hipGetLastError());
    return LABFM_OK;
}

labfm_err weights_fp64(Context* c, const WeightArgs& a, const NodeSet* hs, int32_t* wl, hipStream_t st) {
    int32_t *list = wl, *off, *cnt;
    labfm_err e = build_order_lists(c, a, hs, st, &list, &off, &cnt);
    if (e != LABFM_OK) return e;
    if ((e = weights_invalid_orders(a, list, off, cnt, st)) != LABFM_OK) return e;
    return weights_fp64_lists(c, a, list, off, cnt, ALL_ORDERS, st);
}

}  // namespace labfm
