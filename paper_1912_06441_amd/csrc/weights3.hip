// weights3.hip -- per-node LABFM weights in three dimensions, FP64 (Sec. 3.1
// of King, Lind & Nasar with the third coordinate: p = 3, 9, 19, 34, 55, 83
// for k = 1..6).  Element m is (a, b, c) over total order n = 1..k with a = n..0,
// then b = n-a..0, c = n-a-b; X_m = x^a y^b z^c / (a! b! c!), ABFs of the
// Hermite family H_a(s x) H_b(s y) H_c(s z) phi(|d|).  The node system is
// built and solved as in the two-dimensional FP64 kernel: one wavefront per
// node, M accumulated in registers from basis chunks in LDS, row/column
// equilibration, partial-pivot LU in LDS, FP64 refinement on the moment
// residual, unscaling by h^l (k_weights3, used at k = 5).  At k = 6 the
// system has more elements (83) than a wavefront has lanes: k_weights3w gives
// each lane two rows.  Orders 1..4 run as the two-dimensional FP64 route
// does, in two kernels (k_factor3, k_refine3) with the LU in registers and
// the factors passed through a workspace; the results are the same bit for
// bit.
#include "weights_common.hpp"

namespace labfm {

namespace {

using namespace wk;

constexpr int K3MAX = LABFM_MAX_ORDER3;
constexpr int NM3 = LABFM_MAX_NEIGHBOURS3;  // longest 3-D row
constexpr int p3_of_k(int k) {
    int p = 0;
    for (int m = 2; m <= k + 1; ++m) p += m * (m + 1) / 2;
    return p;
}
constexpr int P3MAX = p3_of_k(K3MAX);  // 83

struct Elem3Table {
    int a[P3MAX], b[P3MAX], c[P3MAX];
};
constexpr Elem3Table make_elems3() {
    Elem3Table t{};
    int m = 0;
    for (int n = 1; n <= K3MAX; ++n)
        for (int a = n; a >= 0; --a)
            for (int b = n - a; b >= 0; --b) {
                t.a[m] = a;
                t.b[m] = b;
                t.c[m] = n - a - b;
                ++m;
            }
    return t;
}
constexpr Elem3Table ELEM3 = make_elems3();

template <int K>
struct Basis3 {
    double px[K + 1], py[K + 1], pz[K + 1];
    double hx[K + 1], hy[K + 1], hz[K + 1];
    double phi;
};

template <int K>
__device__ inline void hermite_row(double t, double (&h)[K + 1]) {
    h[0] = 1.0;
    if (K >= 1) h[1] = 2.0 * t;
#pragma unroll
    for (int e = 1; e < K; ++e) h[e + 1] = 2.0 * t * h[e] - 2.0 * e * h[e - 1];
}

template <int K>
__device__ inline void basis3_prepare(Basis3<K>& B, double dx, double dy, double dz, int rbf, double sigma) {
    B.px[0] = B.py[0] = B.pz[0] = 1.0;
#pragma unroll
    for (int e = 1; e <= K; ++e) {
        B.px[e] = B.px[e - 1] * dx;
        B.py[e] = B.py[e - 1] * dy;
        B.pz[e] = B.pz[e - 1] * dz;
    }
    hermite_row<K>(sigma * dx, B.hx);
    hermite_row<K>(sigma * dy, B.hy);
    hermite_row<K>(sigma * dz, B.hz);
    double F[4];
    rbf_eval(rbf, sqrt(dx * dx + dy * dy + dz * dz), F);
    B.phi = F[0];
}

template <int K>
__device__ inline double monomial3(const Basis3<K>& B, int m) {
    const int a = ELEM3.a[m], b = ELEM3.b[m], c = ELEM3.c[m];
    return B.px[a] * B.py[b] * B.pz[c] * (inv_fact(a) * inv_fact(b) * inv_fact(c));
}

template <int K>
__device__ inline double abf3(const Basis3<K>& B, int m) {
    return B.hx[ELEM3.a[m]] * B.hy[ELEM3.b[m]] * B.hz[ELEM3.c[m]] * B.phi;
}

// 3-D targets: d/dx e1, d/dy e2, d/dz e3, Laplacian e4 + e7 + e9 (1-based)
__device__ inline double target3(unsigned op, int m) {
    switch (op) {
        case LABFM_OP_DX: return m == 0 ? 1.0 : 0.0;
        case LABFM_OP_DY: return m == 1 ? 1.0 : 0.0;
        case LABFM_OP_DZ: return m == 2 ? 1.0 : 0.0;
        case LABFM_OP_LAP: return (m == 3 || m == 6 || m == 8) ? 1.0 : 0.0;
    }
    return 0.0;
}

// M = sum_j X(d_j) W(d_j)^T into sM (row stride P + 1).  Lane (lr, lc) of an
// 8 x 8 grid owns the BS x BS block at (lr BS, lc BS) of the padded matrix;
// the block's rows are accumulated RB at a time (one pass over the basis
// chunks per group of RB rows), which bounds the accumulator registers; CHN
// neighbours per basis chunk.  Each entry sums over j in ascending order
// whatever RB and CHN are.
template <int K, int RB, int CHN = CH>
__device__ inline void assemble3(double* sM, double* sChunk, const double (*sD)[NM3], int N, int rbf, double sigma) {
    constexpr int P = p3_of_k(K);
    constexpr int BS = (P + 7) / 8;
    constexpr int PP = 8 * BS;
    constexpr int LD = P + 1;
    const int lane = threadIdx.x;
    const int lr = lane / 8, lc = lane % 8;
    double* sX = sChunk;
    double* sW = sChunk + CHN * PP;
#pragma unroll
    for (int r0 = 0; r0 < BS; r0 += RB) {
        double acc[RB][BS];
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int c = 0; c < BS; ++c) acc[r][c] = 0.0;
        for (int j0 = 0; j0 < N; j0 += CHN) {
            if (lane < 2 * CHN) {
                const int jj = lane % CHN;
                const int j = j0 + jj;
                double* dst = (lane < CHN ? sX : sW) + jj * PP;
                if (j < N) {
                    Basis3<K> B;
                    basis3_prepare<K>(B, sD[0][j], sD[1][j], sD[2][j], rbf, sigma);
                    if (lane < CHN) {
#pragma unroll
                        for (int m = 0; m < P; ++m) dst[m] = monomial3<K>(B, m);
                    } else {
#pragma unroll
                        for (int m = 0; m < P; ++m) dst[m] = abf3<K>(B, m);
                    }
                } else {
#pragma unroll
                    for (int m = 0; m < P; ++m) dst[m] = 0.0;
                }
#pragma unroll
                for (int m = P; m < PP; ++m) dst[m] = 0.0;
            }
            __syncthreads();
            const int jmax = min(CHN, N - j0);
            for (int jj = 0; jj < jmax; ++jj) {
                double xv[RB], wv[BS];
#pragma unroll
                for (int r = 0; r < RB; ++r) xv[r] = (r0 + r < BS) ? sX[jj * PP + lr * BS + r0 + r] : 0.0;
#pragma unroll
                for (int c = 0; c < BS; ++c) wv[c] = sW[jj * PP + lc * BS + c];
#pragma unroll
                for (int r = 0; r < RB; ++r)
#pragma unroll
                    for (int c = 0; c < BS; ++c) acc[r][c] = fma(xv[r], wv[c], acc[r][c]);
            }
            __syncthreads();
        }
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int c = 0; c < BS; ++c) {
                const int m = lr * BS + r0 + r, nn = lc * BS + c;
                if (r0 + r < BS && m < P && nn < P) sM[m * LD + nn] = acc[r][c];
            }
    }
    __syncthreads();
}

// accumulator rows per pass of assemble3: the whole block up to k = 4, four
// rows at a time above (BS = 7 at k = 5, 11 at k = 6)
constexpr int rb3(int K) { return (p3_of_k(K) + 7) / 8 <= 5 ? (p3_of_k(K) + 7) / 8 : 4; }

struct W3Args {
    const double *x, *y, *z, *R;
    const int64_t* row_ptr;
    const int32_t* col;
    int64_t n, nnz;
    double L[3];
    int per[3];
    int rbf;
    double sigma, tol_stop, tol_pass;
    int max_iters;
    double* w64;
    int8_t* status;
    float* resid;
    int8_t* iters;
};

template <int K>
__global__ __launch_bounds__(64) void k_weights3(W3Args a, OpList ops) {
    constexpr int P = p3_of_k(K);
    constexpr int BS = (P + 7) / 8;
    constexpr int PP = 8 * BS;
    constexpr int LD = P + 1;
    constexpr int JS = NM3 / 64;
    static_assert(P <= 64, "one row per lane");
    // From k = 5 the basis chunks (8 neighbours each) share one buffer with the
    // coefficients and the scaled weights, which are used only after the
    // assembly: 44 KB of LDS per node system, three per CU instead of two.
    constexpr bool SHARE = K >= 5;
    constexpr int CHK = SHARE ? 8 : CH;
    constexpr int NU = SHARE ? cmax(2 * CHK * PP, MAXOPS * NM3 + MAXOPS * PP) : 2 * CH * PP;

    __shared__ double sM[P * LD];
    __shared__ double sU[NU];
    __shared__ double sD[3][NM3];
    __shared__ double sWlA[SHARE ? 1 : MAXOPS * NM3];
    __shared__ double sPsiA[SHARE ? 1 : MAXOPS * PP];
    __shared__ double sRs[P], sCs[P];
    __shared__ int sPerm[P];
    double* const sChunk = sU;
    double (*const sWl)[NM3] = reinterpret_cast<double (*)[NM3]>(SHARE ? sU : sWlA);
    double (*const sPsi)[PP] = reinterpret_cast<double (*)[PP]>(SHARE ? sU + MAXOPS * NM3 : sPsiA);

    const int lane = threadIdx.x;
    const int nops = ops.nops;

    for (int64_t i = blockIdx.x; i < a.n; i += gridDim.x) {
        const int64_t s0 = a.row_ptr[i];
        const int N = (int)(a.row_ptr[i + 1] - s0);
        const double h = 0.5 * a.R[i];
        int status = LABFM_ST_OK;
        double res = INFINITY;
        int iters = 0;
        for (int d = 0; d < nops; ++d)
            if (ops.op[d] == LABFM_OP_LAP && K < 2) status = LABFM_ST_ORDER_TOO_LOW;
        if (status == LABFM_ST_OK && N < P) status = LABFM_ST_TOO_FEW;
        if (status == LABFM_ST_OK && N > NM3) status = LABFM_ST_TOO_MANY;

        double dxr[JS], dyr[JS], dzr[JS];
        if (status == LABFM_ST_OK) {
            const double xi = a.x[i], yi = a.y[i], zi = a.z[i];
#pragma unroll
            for (int js = 0; js < JS; ++js) {
                const int q = lane + 64 * js;
                dxr[js] = dyr[js] = dzr[js] = 0.0;
                if (q < N) {
                    const int32_t j = a.col[s0 + q];
                    dxr[js] = min_image(a.x[j] - xi, a.L[0], a.per[0]) / h;
                    dyr[js] = min_image(a.y[j] - yi, a.L[1], a.per[1]) / h;
                    dzr[js] = min_image(a.z[j] - zi, a.L[2], a.per[2]) / h;
                    sD[0][q] = dxr[js];
                    sD[1][q] = dyr[js];
                    sD[2][q] = dzr[js];
                }
            }
        }
        __syncthreads();

        if (status == LABFM_ST_OK) {
            // ---- assembly: M = sum_j X(d_j) W(d_j)^T, register-blocked
            assemble3<K, rb3(K), CHK>(sM, sChunk, sD, N, a.rbf, a.sigma);

            // ---- equilibration: rows, then columns
            bool sing = false;
            if (lane < P) {
                double mx = 0.0;
                for (int c = 0; c < P; ++c) mx = fmax(mx, fabs(sM[lane * LD + c]));
                if (!(mx > 0.0) || !isfinite(mx)) sing = true;
                const double rs = 1.0 / mx;
                sRs[lane] = rs;
                for (int c = 0; c < P; ++c) sM[lane * LD + c] *= rs;
            }
            __syncthreads();
            if (lane < P) {
                double mx = 0.0;
                for (int r = 0; r < P; ++r) mx = fmax(mx, fabs(sM[r * LD + lane]));
                if (!(mx > 0.0) || !isfinite(mx)) sing = true;
                const double cs = 1.0 / mx;
                sCs[lane] = cs;
                for (int r = 0; r < P; ++r) sM[r * LD + lane] *= cs;
            }
            __syncthreads();
            if (__any(sing)) status = LABFM_ST_SINGULAR;

            // ---- LU with partial pivoting (ties: lowest row)
            int perm = lane;
            if (status == LABFM_ST_OK) {
                for (int kk = 0; kk < P; ++kk) {
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
                        const int pk = __builtin_amdgcn_readlane(perm, kk), pp = __builtin_amdgcn_readlane(perm, pr);
                        if (lane == kk) perm = pp;
                        if (lane == pr) perm = pk;
                    }
                    __syncthreads();
                    // one pass: lane c > kk updates column c of the trailing rows, lane kk
                    // stores the multipliers (every lane reads M[r][kk] before lane kk
                    // overwrites it; rows in groups of eight, loads issued before stores)
                    if (lane >= kk && lane < P) {
                        const double inv = 1.0 / sM[kk * LD + kk];
                        const double u = sM[kk * LD + lane];
                        const bool own = lane == kk;
                        int r = kk + 1;
                        for (; r + 8 <= P; r += 8) {
                            double l[8], a8[8];
#pragma unroll
                            for (int e = 0; e < 8; ++e) {
                                l[e] = sM[(r + e) * LD + kk];
                                a8[e] = sM[(r + e) * LD + lane];
                            }
#pragma unroll
                            for (int e = 0; e < 8; ++e) {
                                const double m = l[e] * inv;
                                sM[(r + e) * LD + lane] = own ? m : fma(-m, u, a8[e]);
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
                for (int d = 0; d < MAXOPS; ++d) b[d] = (d < nops) ? target3(ops.op[d], lane) : 0.0;
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
                    const int q = lane + 64 * js;
#pragma unroll
                    for (int d = 0; d < MAXOPS; ++d) wreg[js][d] = 0.0;
                    if (q < N) {
                        Basis3<K> B;
                        basis3_prepare<K>(B, dxr[js], dyr[js], dzr[js], a.rbf, a.sigma);
#pragma unroll
                        for (int m = 0; m < P; ++m) {
                            const double wm = abf3<K>(B, m);
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
                const int ma = lane < P ? ELEM3.a[lane] : 0;
                const int mb = lane < P ? ELEM3.b[lane] : 0;
                const int mc = lane < P ? ELEM3.c[lane] : 0;
                const double mf = lane < P ? inv_fact(ma) * inv_fact(mb) * inv_fact(mc) : 0.0;
                for (;;) {
                    double r[MAXOPS];
#pragma unroll
                    for (int d = 0; d < MAXOPS; ++d) r[d] = 0.0;
                    if (lane < P) {
                        double accr[MAXOPS];
#pragma unroll
                        for (int d = 0; d < MAXOPS; ++d) accr[d] = 0.0;
                        for (int q = 0; q < N; ++q) {
                            const double dx = sD[0][q], dy = sD[1][q], dz = sD[2][q];
                            double xm = mf;
#pragma unroll
                            for (int e = 0; e < K; ++e) {
                                xm *= (e < ma) ? dx : 1.0;
                                xm *= (e < mb) ? dy : 1.0;
                                xm *= (e < mc) ? dz : 1.0;
                            }
#pragma unroll
                            for (int d = 0; d < MAXOPS; ++d)
                                if (d < nops) accr[d] = fma(xm, sWl[d][q], accr[d]);
                        }
#pragma unroll
                        for (int d = 0; d < MAXOPS; ++d)
                            if (d < nops) r[d] = target3(ops.op[d], lane) - accr[d];
                    }
                    double rm = 0.0;
#pragma unroll
                    for (int d = 0; d < MAXOPS; ++d) {
                        const double ar = fabs(r[d]);
                        rm = (ar > rm || ar != ar) ? ar : rm;
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
                        const int q = lane + 64 * js;
                        if (q < N) {
                            Basis3<K> B;
                            basis3_prepare<K>(B, dxr[js], dyr[js], dzr[js], a.rbf, a.sigma);
                            double dw[MAXOPS];
#pragma unroll
                            for (int d = 0; d < MAXOPS; ++d) dw[d] = 0.0;
#pragma unroll
                            for (int m = 0; m < P; ++m) {
                                const double wm = abf3<K>(B, m);
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
                    const double hl = ops.op[d] == LABFM_OP_LAP ? h * h : h;
#pragma unroll
                    for (int js = 0; js < JS; ++js) {
                        const int q = lane + 64 * js;
                        if (q < N) a.w64[(int64_t)d * a.nnz + s0 + q] = wreg[js][d] / hl;
                    }
                }
            }
        }
        const bool failed = !(status == LABFM_ST_OK || status == LABFM_ST_NOT_CONVERGED);
        if (failed) {
            for (int d = 0; d < nops; ++d)
                for (int q = lane; q < N; q += 64) a.w64[(int64_t)d * a.nnz + s0 + q] = 0.0;
            res = INFINITY;
            iters = 0;
        }
        if (lane == 0) {
            a.status[i] = (int8_t)status;
            if (a.resid) a.resid[i] = (float)res;
            if (a.iters) a.iters[i] = (int8_t)iters;
        }
        __syncthreads();
    }
}

// ---- systems with more elements than lanes (p = 83 at k = 6) --------------
// Lane l holds rows (and columns) l and l + 64.

// Solve M z = b with the equilibrated, pivoted LU in LDS: b[s][d] holds the
// right-hand side of original row lane + 64 s on entry, z[d] of unknown
// lane + 64 s on exit.
template <int P, int LD>
__device__ inline void lu_solve_w(const double* sM, const double* sRs, const double* sCs, const int* sPerm,
                                  double (&b)[2][MAXOPS], int nops) {
    const int lane = threadIdx.x;
    double bs[2][MAXOPS], t[2][MAXOPS];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int m = lane + 64 * s;
        const double rs = m < P ? sRs[m] : 0.0;
#pragma unroll
        for (int d = 0; d < MAXOPS; ++d) bs[s][d] = b[s][d] * rs;
    }
    // position r takes the scaled right-hand side of original row perm[r]
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int r = lane + 64 * s;
        const int src = r < P ? sPerm[r] : 0;
#pragma unroll
        for (int d = 0; d < MAXOPS; ++d) {
            const double v0 = __shfl(bs[0][d], src & 63, 64);
            const double v1 = __shfl(bs[1][d], src & 63, 64);
            t[s][d] = src >= 64 ? v1 : v0;
        }
    }
    // forward: unit lower triangle
    for (int c = 0; c < P - 1; ++c) {
        double l[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int r = lane + 64 * s;
            l[s] = (r > c && r < P) ? sM[r * LD + c] : 0.0;
        }
#pragma unroll
        for (int d = 0; d < MAXOPS; ++d)
            if (d < nops) {
                const double tc = bcast(c < 64 ? t[0][d] : t[1][d], c & 63);
#pragma unroll
                for (int s = 0; s < 2; ++s) t[s][d] -= l[s] * tc;
            }
    }
    // backward
    for (int c = P - 1; c >= 0; --c) {
        const double diag = sM[c * LD + c];
        double u[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int r = lane + 64 * s;
            u[s] = r < c ? sM[r * LD + c] : 0.0;
        }
#pragma unroll
        for (int d = 0; d < MAXOPS; ++d)
            if (d < nops) {
                if (lane == (c & 63)) {
                    if (c < 64)
                        t[0][d] = t[0][d] / diag;
                    else
                        t[1][d] = t[1][d] / diag;
                }
                const double tc = bcast(c < 64 ? t[0][d] : t[1][d], c & 63);
#pragma unroll
                for (int s = 0; s < 2; ++s) t[s][d] -= u[s] * tc;
            }
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int m = lane + 64 * s;
        const double cs = m < P ? sCs[m] : 0.0;
#pragma unroll
        for (int d = 0; d < MAXOPS; ++d) b[s][d] = t[s][d] * cs;
    }
}

template <int K>
__global__ __launch_bounds__(64) void k_weights3w(W3Args a, OpList ops) {
    constexpr int P = p3_of_k(K);
    static_assert(P > 64 && P <= 128, "two rows per lane");
    constexpr int BS = (P + 7) / 8;
    constexpr int PP = 8 * BS;
    constexpr int LD = P + 1;
    constexpr int JS = NM3 / 64;
    // The basis chunks (CHW neighbours each) are needed only during the
    // assembly, the coefficients and the scaled weights only after it: the two
    // share one buffer, which keeps a node system under 80 KB of LDS so that
    // two fit in a CU's 160 KB.
    constexpr int CHW = 10;
    constexpr int NU = cmax(2 * CHW * PP, MAXOPS * NM3 + MAXOPS * PP);

    __shared__ double sM[P * LD];
    __shared__ double sU[NU];
    __shared__ double sD[3][NM3];
    __shared__ double sRs[P], sCs[P];
    __shared__ int sPerm[P];
    double* const sChunk = sU;
    double (*const sWl)[NM3] = reinterpret_cast<double (*)[NM3]>(sU);
    double (*const sPsi)[PP] = reinterpret_cast<double (*)[PP]>(sU + MAXOPS * NM3);

    const int lane = threadIdx.x;
    const int nops = ops.nops;

    for (int64_t i = blockIdx.x; i < a.n; i += gridDim.x) {
        const int64_t s0 = a.row_ptr[i];
        const int N = (int)(a.row_ptr[i + 1] - s0);
        const double h = 0.5 * a.R[i];
        int status = LABFM_ST_OK;
        double res = INFINITY;
        int iters = 0;
        if (status == LABFM_ST_OK && N < P) status = LABFM_ST_TOO_FEW;
        if (status == LABFM_ST_OK && N > NM3) status = LABFM_ST_TOO_MANY;

        double dxr[JS], dyr[JS], dzr[JS];
        if (status == LABFM_ST_OK) {
            const double xi = a.x[i], yi = a.y[i], zi = a.z[i];
#pragma unroll
            for (int js = 0; js < JS; ++js) {
                const int q = lane + 64 * js;
                dxr[js] = dyr[js] = dzr[js] = 0.0;
                if (q < N) {
                    const int32_t j = a.col[s0 + q];
                    dxr[js] = min_image(a.x[j] - xi, a.L[0], a.per[0]) / h;
                    dyr[js] = min_image(a.y[j] - yi, a.L[1], a.per[1]) / h;
                    dzr[js] = min_image(a.z[j] - zi, a.L[2], a.per[2]) / h;
                    sD[0][q] = dxr[js];
                    sD[1][q] = dyr[js];
                    sD[2][q] = dzr[js];
                }
            }
        }
        __syncthreads();

        if (status == LABFM_ST_OK) {
            assemble3<K, rb3(K), CHW>(sM, sChunk, sD, N, a.rbf, a.sigma);

            // ---- equilibration: rows, then columns (lane: rows / columns lane, lane + 64)
            bool sing = false;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int m = lane + 64 * s;
                if (m < P) {
                    double mx = 0.0;
                    for (int c = 0; c < P; ++c) mx = fmax(mx, fabs(sM[m * LD + c]));
                    if (!(mx > 0.0) || !isfinite(mx)) sing = true;
                    const double rs = 1.0 / mx;
                    sRs[m] = rs;
                    for (int c = 0; c < P; ++c) sM[m * LD + c] *= rs;
                }
            }
            __syncthreads();
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int m = lane + 64 * s;
                if (m < P) {
                    double mx = 0.0;
                    for (int r = 0; r < P; ++r) mx = fmax(mx, fabs(sM[r * LD + m]));
                    if (!(mx > 0.0) || !isfinite(mx)) sing = true;
                    const double cs = 1.0 / mx;
                    sCs[m] = cs;
                    for (int r = 0; r < P; ++r) sM[r * LD + m] *= cs;
                }
            }
            __syncthreads();
            if (__any(sing)) status = LABFM_ST_SINGULAR;

            // ---- LU with partial pivoting (ties: lowest row).  Per column: pivot,
            // swap, multipliers stored in place, barrier, trailing update.
            int perm[2] = {lane, lane + 64};
            if (status == LABFM_ST_OK) {
                for (int kk = 0; kk < P; ++kk) {
                    double v[2];
#pragma unroll
                    for (int s = 0; s < 2; ++s) {
                        const int r = lane + 64 * s;
                        v[s] = (r >= kk && r < P) ? fabs(sM[r * LD + kk]) : -1.0;
                    }
                    const double vmax = wave_max_double(fmax(v[0], v[1]));
                    const unsigned long long h0 = __ballot(v[0] == vmax);
                    const unsigned long long h1 = __ballot(v[1] == vmax);
                    if (!(vmax > 0.0) || !isfinite(vmax) || (h0 | h1) == 0ull) {
                        status = LABFM_ST_SINGULAR;
                        break;
                    }
                    const int pr = h0 ? __ffsll((long long)h0) - 1 : 64 + __ffsll((long long)h1) - 1;
                    if (pr != kk) {
#pragma unroll
                        for (int s = 0; s < 2; ++s) {
                            const int c = lane + 64 * s;
                            if (c < P) {
                                const double u = sM[kk * LD + c];
                                sM[kk * LD + c] = sM[pr * LD + c];
                                sM[pr * LD + c] = u;
                            }
                        }
                        const int pk = __builtin_amdgcn_readlane(kk < 64 ? perm[0] : perm[1], kk & 63);
                        const int pp = __builtin_amdgcn_readlane(pr < 64 ? perm[0] : perm[1], pr & 63);
                        if (lane == (kk & 63)) {
                            if (kk < 64)
                                perm[0] = pp;
                            else
                                perm[1] = pp;
                        }
                        if (lane == (pr & 63)) {
                            if (pr < 64)
                                perm[0] = pk;
                            else
                                perm[1] = pk;
                        }
                    }
                    __syncthreads();
                    const double inv = 1.0 / sM[kk * LD + kk];
#pragma unroll
                    for (int s = 0; s < 2; ++s) {
                        const int r = lane + 64 * s;
                        if (r > kk && r < P) sM[r * LD + kk] = sM[r * LD + kk] * inv;
                    }
                    __syncthreads();
#pragma unroll
                    for (int s = 0; s < 2; ++s) {
                        const int c = lane + 64 * s;
                        if (c > kk && c < P) {
                            const double u = sM[kk * LD + c];
                            for (int r = kk + 1; r < P; ++r) sM[r * LD + c] = fma(-sM[r * LD + kk], u, sM[r * LD + c]);
                        }
                    }
                    __syncthreads();
                }
            }
#pragma unroll
            for (int s = 0; s < 2; ++s)
                if (lane + 64 * s < P) sPerm[lane + 64 * s] = perm[s];
            __syncthreads();

            if (status == LABFM_ST_OK) {
                // ---- initial solve
                double b[2][MAXOPS];
#pragma unroll
                for (int s = 0; s < 2; ++s)
#pragma unroll
                    for (int d = 0; d < MAXOPS; ++d) b[s][d] = (d < nops) ? target3(ops.op[d], lane + 64 * s) : 0.0;
                lu_solve_w<P, LD>(sM, sRs, sCs, sPerm, b, nops);
#pragma unroll
                for (int s = 0; s < 2; ++s)
                    if (lane + 64 * s < P)
#pragma unroll
                        for (int d = 0; d < MAXOPS; ++d)
                            if (d < nops) sPsi[d][lane + 64 * s] = b[s][d];
                __syncthreads();

                // ---- w_j = W(d_j) . Psi
                double wreg[JS][MAXOPS];
#pragma unroll
                for (int js = 0; js < JS; ++js) {
                    const int q = lane + 64 * js;
#pragma unroll
                    for (int d = 0; d < MAXOPS; ++d) wreg[js][d] = 0.0;
                    if (q < N) {
                        Basis3<K> B;
                        basis3_prepare<K>(B, dxr[js], dyr[js], dzr[js], a.rbf, a.sigma);
#pragma unroll
                        for (int m = 0; m < P; ++m) {
                            const double wm = abf3<K>(B, m);
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
                int ma[2], mb[2], mc[2];
                double mf[2];
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const int m = lane + 64 * s;
                    ma[s] = m < P ? ELEM3.a[m] : 0;
                    mb[s] = m < P ? ELEM3.b[m] : 0;
                    mc[s] = m < P ? ELEM3.c[m] : 0;
                    mf[s] = m < P ? inv_fact(ma[s]) * inv_fact(mb[s]) * inv_fact(mc[s]) : 0.0;
                }
                for (;;) {
                    double r[2][MAXOPS];
                    double rm = 0.0;
#pragma unroll
                    for (int s = 0; s < 2; ++s) {
                        const int m = lane + 64 * s;
#pragma unroll
                        for (int d = 0; d < MAXOPS; ++d) r[s][d] = 0.0;
                        if (m < P) {
                            double accr[MAXOPS];
#pragma unroll
                            for (int d = 0; d < MAXOPS; ++d) accr[d] = 0.0;
                            for (int q = 0; q < N; ++q) {
                                const double dx = sD[0][q], dy = sD[1][q], dz = sD[2][q];
                                double xm = mf[s];
#pragma unroll
                                for (int e = 0; e < K; ++e) {
                                    xm *= (e < ma[s]) ? dx : 1.0;
                                    xm *= (e < mb[s]) ? dy : 1.0;
                                    xm *= (e < mc[s]) ? dz : 1.0;
                                }
#pragma unroll
                                for (int d = 0; d < MAXOPS; ++d)
                                    if (d < nops) accr[d] = fma(xm, sWl[d][q], accr[d]);
                            }
#pragma unroll
                            for (int d = 0; d < MAXOPS; ++d)
                                if (d < nops) r[s][d] = target3(ops.op[d], m) - accr[d];
                        }
#pragma unroll
                        for (int d = 0; d < MAXOPS; ++d) {
                            const double ar = fabs(r[s][d]);
                            rm = (ar > rm || ar != ar) ? ar : rm;
                        }
                    }
                    if (!isfinite(rm)) rm = INFINITY;
                    res = wave_max(rm);
                    if (!(res > a.tol_stop) || iters >= a.max_iters) break;
                    lu_solve_w<P, LD>(sM, sRs, sCs, sPerm, r, nops);
                    __syncthreads();
#pragma unroll
                    for (int s = 0; s < 2; ++s)
                        if (lane + 64 * s < P)
#pragma unroll
                            for (int d = 0; d < MAXOPS; ++d)
                                if (d < nops) sPsi[d][lane + 64 * s] = r[s][d];
                    __syncthreads();
#pragma unroll
                    for (int js = 0; js < JS; ++js) {
                        const int q = lane + 64 * js;
                        if (q < N) {
                            Basis3<K> B;
                            basis3_prepare<K>(B, dxr[js], dyr[js], dzr[js], a.rbf, a.sigma);
                            double dw[MAXOPS];
#pragma unroll
                            for (int d = 0; d < MAXOPS; ++d) dw[d] = 0.0;
#pragma unroll
                            for (int m = 0; m < P; ++m) {
                                const double wm = abf3<K>(B, m);
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
                    const double hl = ops.op[d] == LABFM_OP_LAP ? h * h : h;
#pragma unroll
                    for (int js = 0; js < JS; ++js) {
                        const int q = lane + 64 * js;
                        if (q < N) a.w64[(int64_t)d * a.nnz + s0 + q] = wreg[js][d] / hl;
                    }
                }
            }
        }
        const bool failed = !(status == LABFM_ST_OK || status == LABFM_ST_NOT_CONVERGED);
        if (failed) {
            for (int d = 0; d < nops; ++d)
                for (int q = lane; q < N; q += 64) a.w64[(int64_t)d * a.nnz + s0 + q] = 0.0;
            res = INFINITY;
            iters = 0;
        }
        if (lane == 0) {
            a.status[i] = (int8_t)status;
            if (a.resid) a.resid[i] = (float)res;
            if (a.iters) a.iters[i] = (int8_t)iters;
        }
        __syncthreads();
    }
}

// ---- orders 1..4 in two kernels ----------------------------------------
// The same node systems, steps and roundings as k_weights3, split as the
// two-dimensional FP64 route is: k_factor3 (assembly, equilibration, LU with
// one row per lane in registers, first solve) hands each node's factors
// (column-major by pivot place), scales, places, Psi and status through a
// workspace to k_refine3 (weights, FP64 moment residual, refinement), which
// loads a node's LU rows straight into registers when it needs a correction.

struct Factor3Ws {
    double* lu;     // [slots][P * P]: entry (r, c) at c * P + r, rows by place
    double* rs;     // [slots][P]
    double* cs;     // [slots][P]
    double* psi;    // [slots][MAXOPS][P]
    int32_t* perm;  // [slots][P]: the row (of the equilibrated M) at each place
    int8_t* st;     // [slots]
};

// Operator slots 0..NB3-1 are always computed, on zero coefficients when a
// call asks for fewer; slots beyond follow the run-time count (a fourth slot
// costs more in registers than its branches do).
constexpr int NB3 = 3;
__device__ inline bool live3(int d, int nops) { return d < NB3 || d < nops; }

// v of another lane of the same row of 16 (CTRL 0x121..0x12f: rotate right)
template <int CTRL>
__device__ inline double dpp3(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
// maximum over the wavefront: rotations by 8, 4, 2, 1 lanes, then the four row maxima
__device__ inline double wave_max3(double v) {
    v = fmax(v, dpp3<0x128>(v));
    v = fmax(v, dpp3<0x124>(v));
    v = fmax(v, dpp3<0x122>(v));
    v = fmax(v, dpp3<0x121>(v));
    return fmax(fmax(bcast(v, 0), bcast(v, 16)), fmax(bcast(v, 32), bcast(v, 48)));
}

template <int K>
__global__ __launch_bounds__(64) void k_factor3(W3Args a, OpList ops, int64_t begin, int64_t end, Factor3Ws w) {
    constexpr int P = p3_of_k(K);
    constexpr int BS = (P + 7) / 8;
    constexpr int PP = 8 * BS;
    constexpr int LD = P + 1;
    constexpr int CHK = K >= 5 ? 8 : CH;
    static_assert(P <= 64, "one row per lane");
    // one pass of the assembly over the chunks (all accumulator rows at once):
    // the chunks are read only before M is written, so they share its buffer
    constexpr bool ALIAS = rb3(K) >= BS;
    __shared__ double sMC[ALIAS ? cmax(P * LD, 2 * CHK * PP) : P * LD];
    __shared__ double sCh[ALIAS ? 1 : 2 * CHK * PP];
    double* const sM = sMC;
    double* const sChunk = ALIAS ? sMC : sCh;
    __shared__ double sD[3][NM3];
    __shared__ double sRs[P], sCs[P];
    __shared__ int sPerm[P];

    const int lane = threadIdx.x;
    const int nops = ops.nops;

    for (int64_t i = begin + blockIdx.x; i < end; i += gridDim.x) {
        const int64_t slot = i - begin;
        const int64_t s0 = a.row_ptr[i];
        const int N = (int)(a.row_ptr[i + 1] - s0);
        const double h = 0.5 * a.R[i];
        int status = LABFM_ST_OK;
        for (int d = 0; d < nops; ++d)
            if (ops.op[d] == LABFM_OP_LAP && K < 2) status = LABFM_ST_ORDER_TOO_LOW;
        if (status == LABFM_ST_OK && N < P) status = LABFM_ST_TOO_FEW;
        if (status == LABFM_ST_OK && N > NM3) status = LABFM_ST_TOO_MANY;

        if (status == LABFM_ST_OK) {
            const double xi = a.x[i], yi = a.y[i], zi = a.z[i];
            for (int q = lane; q < N; q += 64) {
                const int32_t j = a.col[s0 + q];
                sD[0][q] = min_image(a.x[j] - xi, a.L[0], a.per[0]) / h;
                sD[1][q] = min_image(a.y[j] - yi, a.L[1], a.per[1]) / h;
                sD[2][q] = min_image(a.z[j] - zi, a.L[2], a.per[2]) / h;
            }
        }
        __syncthreads();

        if (status == LABFM_ST_OK) {
            // ---- assembly: M = sum_j X(d_j) W(d_j)^T
            assemble3<K, rb3(K), CHK>(sM, sChunk, sD, N, a.rbf, a.sigma);

            // ---- equilibration: rows, then columns
            bool sing = false;
            if (lane < P) {
                double mx = 0.0;
                for (int c = 0; c < P; ++c) mx = fmax(mx, fabs(sM[lane * LD + c]));
                if (!(mx > 0.0) || !isfinite(mx)) sing = true;
                const double rs = 1.0 / mx;
                sRs[lane] = rs;
                for (int c = 0; c < P; ++c) sM[lane * LD + c] *= rs;
            }
            __syncthreads();
            if (lane < P) {
                double mx = 0.0;
                for (int r = 0; r < P; ++r) mx = fmax(mx, fabs(sM[r * LD + lane]));
                if (!(mx > 0.0) || !isfinite(mx)) sing = true;
                const double cs = 1.0 / mx;
                sCs[lane] = cs;
                for (int r = 0; r < P; ++r) sM[r * LD + lane] *= cs;
            }
            __syncthreads();
            if (__any(sing)) status = LABFM_ST_SINGULAR;

            // ---- LU with partial pivoting, row r in lane r's registers; pos is
            // the row's place in the pivoted order (ties: the lowest place)
            double row[P];
#pragma unroll
            for (int c = 0; c < P; ++c) row[c] = lane < P ? sM[lane * LD + c] : 0.0;
            int pos = lane;
            if (status == LABFM_ST_OK) {
#pragma unroll
                for (int kk = 0; kk < P; ++kk) {
                    const double v = (pos >= kk && pos < P) ? fabs(row[kk]) : -1.0;
                    const double vmax = wave_max3(v);
                    const unsigned long long hit = __ballot(v == vmax);
                    if (!(vmax > 0.0) || !isfinite(vmax) || hit == 0ull) {
                        status = LABFM_ST_SINGULAR;
                        break;
                    }
                    int pl = __ffsll((long long)hit) - 1;
                    if (__popcll(hit) > 1) {
                        int cand = v == vmax ? pos : 1 << 20;
#pragma unroll
                        for (int off = 32; off >= 1; off >>= 1) cand = min(cand, __shfl_xor(cand, off, 64));
                        pl = __ffsll((long long)__ballot(pos == cand)) - 1;
                    }
                    const int ppos = __builtin_amdgcn_readlane(pos, pl);
                    pos = lane == pl ? kk : (pos == kk ? ppos : pos);
                    const double inv = 1.0 / bcast(row[kk], pl);
                    const bool upd = pos > kk && pos < P;
                    const double m = row[kk] * inv;
#pragma unroll
                    for (int c0 = kk + 1; c0 < P; c0 += 4) {
                        double u[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            if (c0 + q < P) u[q] = bcast(row[c0 + q], pl);
                        if (upd) {
#pragma unroll
                            for (int q = 0; q < 4; ++q)
                                if (c0 + q < P) row[c0 + q] = fma(-m, u[q], row[c0 + q]);
                        }
                    }
                    if (upd) row[kk] = m;
                }
            }
            if (lane < P) sPerm[pos] = lane;
            __syncthreads();
            if (status == LABFM_ST_OK) {
                // ---- first solve, in places; the row at place c is in lane perm_reg of lane c
                double t[MAXOPS];
                const double rs = lane < P ? sRs[lane] : 0.0;
#pragma unroll
                for (int d = 0; d < MAXOPS; ++d) t[d] = ((d < nops) ? target3(ops.op[d], lane) : 0.0) * rs;
                const int perm_reg = lane < P ? sPerm[lane] : 0;
#pragma unroll
                for (int c = 0; c < P - 1; ++c) {
                    const int src = __builtin_amdgcn_readlane(perm_reg, c);
                    const double l = (pos > c && pos < P) ? row[c] : 0.0;
#pragma unroll
                    for (int d = 0; d < MAXOPS; ++d)
                        if (live3(d, nops)) t[d] -= l * bcast(t[d], src);
                }
#pragma unroll
                for (int c = P - 1; c >= 0; --c) {
                    const int src = __builtin_amdgcn_readlane(perm_reg, c);
                    const double u = pos < c ? row[c] : 0.0;
#pragma unroll
                    for (int d = 0; d < MAXOPS; ++d) {
                        if (live3(d, nops)) {
                            const double q = t[d] / row[c];  // every lane divides; lane src keeps it
                            t[d] = lane == src ? q : t[d];
                            t[d] -= u * bcast(t[d], src);
                        }
                    }
                }
                const int from = lane < P ? sPerm[lane] : 0;
                const double cs = lane < P ? sCs[lane] : 0.0;
#pragma unroll
                for (int d = 0; d < MAXOPS; ++d) {
                    const double z = __shfl(t[d], from, 64) * cs;
                    if (lane < P && d < nops) w.psi[(slot * MAXOPS + d) * (int64_t)P + lane] = z;
                }
                double* lu = w.lu + slot * (int64_t)(P * P);
                if (lane < P) {
#pragma unroll
                    for (int c = 0; c < P; ++c) lu[c * P + pos] = row[c];
                    w.rs[slot * (int64_t)P + lane] = rs;
                    w.cs[slot * (int64_t)P + lane] = cs;
                    w.perm[slot * (int64_t)P + lane] = sPerm[lane];
                }
            }
        }
        if (lane == 0) w.st[slot] = (int8_t)status;
        __syncthreads();
    }
}

// Solve M z = b with one node's factors from the workspace: lane r loads row r
// (one contiguous load per column of the column-major store) and the solve
// runs in registers; the arithmetic and its order are lu_solve's.
template <int P>
__device__ inline void lu_solve_rows3(const double* lu_node, double rs, double cs, int pr, double (&b)[MAXOPS],
                                      int nops) {
    const int lane = threadIdx.x;
    // the base pointer passes through an empty asm so that the column
    // addresses are formed here instead of being held across the caller's loop
    uint64_t bits = (uint64_t)lu_node;
    asm volatile("" : "+s"(bits));
    const double* lu = (const double*)bits;
    double t[MAXOPS];
#pragma unroll
    for (int d = 0; d < MAXOPS; ++d) t[d] = __shfl(b[d] * rs, pr, 64);
    double row[P];
#pragma unroll
    for (int c = 0; c < P - 1; ++c) row[c] = (lane > c && lane < P) ? lu[c * P + lane] : 0.0;
#pragma unroll
    for (int c = 0; c < P - 1; ++c)
#pragma unroll
        for (int d = 0; d < MAXOPS; ++d)
            if (live3(d, nops)) t[d] -= row[c] * bcast(t[d], c);
#pragma unroll
    for (int c = 0; c < P; ++c) row[c] = (lane <= c) ? lu[c * P + lane] : 0.0;
#pragma unroll
    for (int c = P - 1; c >= 0; --c) {
        const double u = lane < c ? row[c] : 0.0;
#pragma unroll
        for (int d = 0; d < MAXOPS; ++d) {
            if (live3(d, nops)) {
                const double q = t[d] / row[c];  // every lane divides; lane c keeps it
                t[d] = lane == c ? q : t[d];
                t[d] -= u * bcast(t[d], c);
            }
        }
    }
#pragma unroll
    for (int d = 0; d < MAXOPS; ++d) b[d] = t[d] * cs;
}

template <int K>
__global__ __launch_bounds__(64) void k_refine3(W3Args a, OpList ops, int64_t begin, int64_t end, Factor3Ws w) {
    constexpr int P = p3_of_k(K);
    constexpr int BS = (P + 7) / 8;
    constexpr int PP = 8 * BS;
    __shared__ double sD[3][NM3];
    __shared__ double sWl[MAXOPS][NM3];  // scaled weights: running sums, and the residual's input
    __shared__ double sPsi[MAXOPS][PP];

    const int lane = threadIdx.x;
    const int nops = ops.nops;

    for (int64_t i = begin + blockIdx.x; i < end; i += gridDim.x) {
        const int64_t slot = i - begin;
        const int64_t s0 = a.row_ptr[i];
        const int N = (int)(a.row_ptr[i + 1] - s0);
        const double h = 0.5 * a.R[i];
        int status = w.st[slot];
        double res = INFINITY;
        int iters = 0;

        if (status == LABFM_ST_OK) {
            const double xi = a.x[i], yi = a.y[i], zi = a.z[i];
            for (int q = lane; q < N; q += 64) {
                const int32_t j = a.col[s0 + q];
                sD[0][q] = min_image(a.x[j] - xi, a.L[0], a.per[0]) / h;
                sD[1][q] = min_image(a.y[j] - yi, a.L[1], a.per[1]) / h;
                sD[2][q] = min_image(a.z[j] - zi, a.L[2], a.per[2]) / h;
            }
            if (lane < P)
                for (int d = 0; d < MAXOPS; ++d)
                    if (live3(d, nops)) sPsi[d][lane] = d < nops ? w.psi[(slot * MAXOPS + d) * (int64_t)P + lane] : 0.0;
        }
        __syncthreads();

        if (status == LABFM_ST_OK) {
            // ---- w_j = W(d_j) . Psi (lane q keeps neighbour q's sums in sWl)
            for (int q = lane; q < N; q += 64) {
                asm volatile("" ::: "memory");  // keeps Psi's loads inside the loop
                double wv[MAXOPS];
#pragma unroll
                for (int d = 0; d < MAXOPS; ++d) wv[d] = 0.0;
                Basis3<K> B;
                basis3_prepare<K>(B, sD[0][q], sD[1][q], sD[2][q], a.rbf, a.sigma);
#pragma unroll
                for (int m = 0; m < P; ++m) {
                    const double wm = abf3<K>(B, m);
#pragma unroll
                    for (int d = 0; d < MAXOPS; ++d)
                        if (live3(d, nops)) wv[d] = fma(wm, sPsi[d][m], wv[d]);
                }
#pragma unroll
                for (int d = 0; d < MAXOPS; ++d)
                    if (live3(d, nops)) sWl[d][q] = wv[d];
            }
            __syncthreads();

            const double* lu = w.lu + slot * (int64_t)(P * P);
            double rs = 0.0, cs = 0.0;
            int pr = 0;
            bool lu_in = false;

            // ---- refinement on the moment residual (FP64)
            const int ma = lane < P ? ELEM3.a[lane] : 0;
            const int mb = lane < P ? ELEM3.b[lane] : 0;
            const int mc = lane < P ? ELEM3.c[lane] : 0;
            const double mf = lane < P ? inv_fact(ma) * inv_fact(mb) * inv_fact(mc) : 0.0;
            for (;;) {
                double r[MAXOPS];
#pragma unroll
                for (int d = 0; d < MAXOPS; ++d) r[d] = 0.0;
                if (lane < P) {
                    double accr[MAXOPS];
#pragma unroll
                    for (int d = 0; d < MAXOPS; ++d) accr[d] = 0.0;
                    // every slot's sums are read without a branch (a slot beyond the
                    // operator count is never used); four neighbours loaded ahead
#pragma unroll 4
                    for (int q = 0; q < N; ++q) {
                        const double dx = sD[0][q], dy = sD[1][q], dz = sD[2][q];
                        double wq[MAXOPS];
#pragma unroll
                        for (int d = 0; d < MAXOPS; ++d) wq[d] = sWl[d][q];
                        double xm = mf;
#pragma unroll
                        for (int e = 0; e < K; ++e) {
                            xm *= (e < ma) ? dx : 1.0;
                            xm *= (e < mb) ? dy : 1.0;
                            xm *= (e < mc) ? dz : 1.0;
                        }
#pragma unroll
                        for (int d = 0; d < MAXOPS; ++d) accr[d] = fma(xm, wq[d], accr[d]);
                    }
#pragma unroll
                    for (int d = 0; d < MAXOPS; ++d)
                        if (d < nops) r[d] = target3(ops.op[d], lane) - accr[d];
                }
                double rm = 0.0;
#pragma unroll
                for (int d = 0; d < MAXOPS; ++d) {
                    const double ar = fabs(r[d]);
                    rm = (ar > rm || ar != ar) ? ar : rm;
                }
                if (!isfinite(rm)) rm = INFINITY;
                res = wave_max(rm);
                if (!(res > a.tol_stop) || iters >= a.max_iters) break;
                if (!lu_in) {
                    if (lane < P) {
                        rs = w.rs[slot * (int64_t)P + lane];
                        cs = w.cs[slot * (int64_t)P + lane];
                        pr = w.perm[slot * (int64_t)P + lane];
                    }
                    lu_in = true;
                }
                lu_solve_rows3<P>(lu, rs, cs, pr, r, nops);
                if (lane < P)
#pragma unroll
                    for (int d = 0; d < MAXOPS; ++d)
                        if (live3(d, nops)) sPsi[d][lane] = r[d];
                __syncthreads();
                for (int q = lane; q < N; q += 64) {
                    asm volatile("" ::: "memory");
                    Basis3<K> B;
                    basis3_prepare<K>(B, sD[0][q], sD[1][q], sD[2][q], a.rbf, a.sigma);
                    double dw[MAXOPS];
#pragma unroll
                    for (int d = 0; d < MAXOPS; ++d) dw[d] = 0.0;
#pragma unroll
                    for (int m = 0; m < P; ++m) {
                        const double wm = abf3<K>(B, m);
#pragma unroll
                        for (int d = 0; d < MAXOPS; ++d)
                            if (live3(d, nops)) dw[d] = fma(wm, sPsi[d][m], dw[d]);
                    }
#pragma unroll
                    for (int d = 0; d < MAXOPS; ++d)
                        if (live3(d, nops)) sWl[d][q] += dw[d];
                }
                __syncthreads();
                ++iters;
            }
            if (!(res <= a.tol_pass)) status = LABFM_ST_NOT_CONVERGED;

            // ---- unscale and store
            for (int d = 0; d < nops; ++d) {
                const double hl = ops.op[d] == LABFM_OP_LAP ? h * h : h;
                for (int q = lane; q < N; q += 64) a.w64[(int64_t)d * a.nnz + s0 + q] = sWl[d][q] / hl;
            }
        }
        const bool failed = !(status == LABFM_ST_OK || status == LABFM_ST_NOT_CONVERGED);
        if (failed) {
            for (int d = 0; d < nops; ++d)
                for (int q = lane; q < N; q += 64) a.w64[(int64_t)d * a.nnz + s0 + q] = 0.0;
            res = INFINITY;
            iters = 0;
        }
        if (lane == 0) {
            a.status[i] = (int8_t)status;
            if (a.resid) a.resid[i] = (float)res;
            if (a.iters) a.iters[i] = (int8_t)iters;
        }
        __syncthreads();
    }
}

template <typename Kern>
int grid3_of(Kern kern) {
    int dev = 0, ncu = 0, per = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, 64, 0);
    if (ncu <= 0) ncu = 256;
    if (per <= 0) per = 1;
    return ncu * per;
}

template <int K>
int grid3_for() {
    static int g = 0;
    if (g == 0) g = grid3_of(k_weights3<K>);
    return g;
}
template <int K>
int grid3w_for() {
    static int g = 0;
    if (g == 0) g = grid3_of(k_weights3w<K>);
    return g;
}

template <int K>
void launch3(const W3Args& a, const OpList& ops, hipStream_t st) {
    k_weights3<K><<<grid3_for<K>(), 64, 0, st>>>(a, ops);
}
template <int K>
void launch3w(const W3Args& a, const OpList& ops, hipStream_t st) {
    k_weights3w<K><<<grid3w_for<K>(), 64, 0, st>>>(a, ops);
}

// node slots of the factor workspace: one chunk of nodes at a time
constexpr int64_t FACTOR3_SLOTS = 1 << 18;

template <int K>
size_t factor3_bytes(int64_t slots) {
    constexpr int64_t P = p3_of_k(K);
    return sizeof(double) * (size_t)(slots * (P * P + 2 * P + MAXOPS * P)) + sizeof(int32_t) * (size_t)(slots * P) +
           (size_t)slots;
}

template <int K>
labfm_err launch3_split(Context* c, const W3Args& a, const OpList& ops, hipStream_t st) {
    constexpr int64_t P = p3_of_k(K);
    static int gf = 0, gr = 0;
    if (gf == 0) gf = grid3_of(k_factor3<K>);
    if (gr == 0) gr = grid3_of(k_refine3<K>);
    const int64_t slots = a.n < FACTOR3_SLOTS ? a.n : FACTOR3_SLOTS;
    labfm_err e = ensure(c->factors3, factor3_bytes<K>(slots));
    if (e != LABFM_OK) return e;
    char* base = (char*)c->factors3.p;
    Factor3Ws w;
    w.lu = (double*)base;
    w.rs = w.lu + slots * P * P;
    w.cs = w.rs + slots * P;
    w.psi = w.cs + slots * P;
    w.perm = (int32_t*)(w.psi + slots * MAXOPS * P);
    w.st = (int8_t*)(w.perm + slots * P);
    for (int64_t b0 = 0; b0 < a.n; b0 += slots) {
        const int64_t end = b0 + slots < a.n ? b0 + slots : a.n;
        k_factor3<K><<<gf, 64, 0, st>>>(a, ops, b0, end, w);
        k_refine3<K><<<gr, 64, 0, st>>>(a, ops, b0, end, w);
    }
    return LABFM_OK;
}

}  // namespace

labfm_err weights3(Context* c, const double* x, const double* y, const double* z, int64_t n, const Grid3& g,
                   const double* R, int k, const int64_t* row_ptr, const int32_t* col, int64_t nnz,
                   const labfm_wopts* opt, double* w64, int8_t* status, float* resid, int8_t* iters,
                   hipStream_t st) {
    if (n == 0) return LABFM_OK;
    W3Args a{};
    a.x = x;
    a.y = y;
    a.z = z;
    a.R = R;
    a.row_ptr = row_ptr;
    a.col = col;
    a.n = n;
    a.nnz = nnz;
    for (int d = 0; d < 3; ++d) {
        a.L[d] = g.L[d];
        a.per[d] = g.per[d];
    }
    a.rbf = opt->rbf;
    a.sigma = opt->sigma;
    a.tol_stop = opt->tol_stop;
    a.tol_pass = opt->tol_pass;
    a.max_iters = opt->max_iters;
    a.w64 = w64;
    a.status = status;
    a.resid = resid;
    a.iters = iters;
    OpList ops{};
    ops.nops = 0;
    for (int b = 0; b < 6; ++b)
        if (opt->ops & (1u << b)) ops.op[ops.nops++] = 1u << b;
    static const char* names[K3MAX + 1] = {"",           "weights3d_k1", "weights3d_k2", "weights3d_k3",
                                           "weights3d_k4", "weights3d_k5", "weights3d_k6"};
    // orders 1..4: the two-kernel route.  Order 5 keeps the single kernel: its
    // 55 rows in registers spill, and the pair took 17.7 ms at 32^3 against
    // 10.4 ms.  Order 6 (83 elements, two rows per lane): one kernel.
    KernelTimer timer(c, names[k], st);
    labfm_err e = LABFM_OK;
    switch (k) {
        case 1: e = launch3_split<1>(c, a, ops, st); break;
        case 2: e = launch3_split<2>(c, a, ops, st); break;
        case 3: e = launch3_split<3>(c, a, ops, st); break;
        case 4: e = launch3_split<4>(c, a, ops, st); break;
        case 5: launch3<5>(a, ops, st); break;
        default: launch3w<6>(a, ops, st); break;
    }
    if (e != LABFM_OK) return e;
    LABFM_HIP_CHECK(hipGetLastError());
    return LABFM_OK;
}

}  // namespace labfm
