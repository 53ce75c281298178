// weights_mixed.hip -- per-node LABFM weights, mixed precision.
//
// Same system as the FP64 path (Sec. 3.1 of King, Lind & Nasar: M = sum_j
// X(d_j) W(d_j)^T, M Psi = C, w = W Psi), with the work split by precision:
//   * basis values rounded to FP32 and M assembled on the matrix cores
//     (v_mfma_f32_16x16x4f32, FP32 accumulation),
//   * FP32 equilibration and LU with partial pivoting in LDS,
//   * FP64 weights w = W Psi, FP64 moment residual r = C - X^T w and FP64
//     weight refinement w += W (M32^-1 r) until ||r|| <= tol_stop.
// Nodes whose refinement does not reach tol_pass are appended to a per-order
// retry list and recomputed by the FP64 kernels.  With a warm start (psi0),
// nodes of that order begin the refinement from W Psi0 instead of from a
// first solve with the FP32 factors.
//
// Launch shape: one 64-lane wavefront per node system, persistent over the
// per-order work list.  M tiles: lane l of the 16x16x4 MFMA holds A[l%16][l/16]
// and B[l/16][l%16]; the 16x16 result lane l, register i is row 4(l/16)+i,
// column l%16.
#include "weights_common.hpp"

namespace labfm {

namespace {
using namespace wk;

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int CHM = 16;  // neighbours per basis chunk (four MFMA k-steps)

template <int K, int FAM>
__global__ __launch_bounds__(64) void k_weights_mixed(WeightArgs a, OpList ops, const int32_t* list,
                                                      const int32_t* list_off, const int32_t* list_cnt,
                                                      int32_t* retry_list, int32_t* retry_cnt) {
    constexpr int P = p_of_k(K);
    constexpr int T = (P + 15) / 16;  // MFMA tiles per dimension
    constexpr int PP = 16 * T;
    constexpr int LD = P + 1;
    constexpr int JS = NMAX / 64;

    __shared__ float sM[cmax(P * LD, 2 * CHM * PP)];  // M / LU factors, aliased with the FP32 basis chunk
    __shared__ double sD[2][NMAX];
    __shared__ double sWl[MAXOPS][NMAX];
    __shared__ double sPsi[MAXOPS][PP];
    __shared__ float sRs[P], sCs[P];
    __shared__ int sPerm[P];

    const int lane = threadIdx.x;
    const int nops = ops.nops;
    const int count = list_cnt[K];
    const int32_t* mylist = list + list_off[K];

    for (int t = blockIdx.x; t < count; t += gridDim.x) {
        const int32_t g = mylist[t];
        NodeSet S;
        int64_t i;
        resolve(a, g, S, i);
        const int64_t s0 = S.row_ptr[i];
        const int N = (int)(S.row_ptr[i + 1] - s0);
        const double h = 0.5 * S.R[i];
        int status = LABFM_ST_OK;
        double res = INFINITY;
        int iters = 0;

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
                const int q = lane + 64 * js;
                dxr[js] = 0.0;
                dyr[js] = 0.0;
                if (q < N) {
                    const int32_t j = S.col[s0 + q];
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
            // ---- assembly on the matrix cores: M = X^T W, K-dimension = neighbours
            floatx4 acc[T][T];
#pragma unroll
            for (int ti = 0; ti < T; ++ti)
#pragma unroll
                for (int tj = 0; tj < T; ++tj) acc[ti][tj] = floatx4{0.f, 0.f, 0.f, 0.f};
            float* sX = sM;
            float* sW = sM + CHM * PP;
            for (int j0 = 0; j0 < N; j0 += CHM) {
                if (lane < 2 * CHM) {
                    const int jj = lane % CHM;
                    const int j = j0 + jj;
                    float* dst = (lane < CHM ? sX : sW) + jj * PP;
                    if (j < N) {
                        BasisState<K> B;
                        basis_prepare<K, FAM>(B, sD[0][j], sD[1][j], a.rbf, a.sigma);
                        if (lane < CHM) {
#pragma unroll
                            for (int m = 0; m < P; ++m) dst[m] = (float)monomial<K>(B, m);
                        } else {
#pragma unroll
                            for (int m = 0; m < P; ++m) dst[m] = (float)abf<K, FAM>(B, m);
                        }
                    } else {
#pragma unroll
                        for (int m = 0; m < P; ++m) dst[m] = 0.f;
                    }
#pragma unroll
                    for (int m = P; m < PP; ++m) dst[m] = 0.f;
                }
                __syncthreads();
#pragma unroll
                for (int ks = 0; ks < CHM / 4; ++ks) {
                    const int jb = ks * 4 + lane / 16;
                    float av[T], bv[T];
#pragma unroll
                    for (int ti = 0; ti < T; ++ti) av[ti] = sX[jb * PP + 16 * ti + lane % 16];
#pragma unroll
                    for (int tj = 0; tj < T; ++tj) bv[tj] = sW[jb * PP + 16 * tj + lane % 16];
#pragma unroll
                    for (int ti = 0; ti < T; ++ti)
#pragma unroll
                        for (int tj = 0; tj < T; ++tj)
                            acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ti], bv[tj], acc[ti][tj], 0, 0, 0);
                }
                __syncthreads();
            }
#pragma unroll
            for (int ti = 0; ti < T; ++ti)
#pragma unroll
                for (int tj = 0; tj < T; ++tj)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int m = 16 * ti + 4 * (lane / 16) + e, nn = 16 * tj + lane % 16;
                        if (m < P && nn < P) sM[m * LD + nn] = acc[ti][tj][e];
                    }
            __syncthreads();

            // ---- FP32 equilibration
            bool sing = false;
            if (lane < P) {
                float mx = 0.f;
                for (int c = 0; c < P; ++c) mx = fmaxf(mx, fabsf(sM[lane * LD + c]));
                if (!(mx > 0.f) || !isfinite(mx)) sing = true;
                const float rs = 1.f / mx;
                sRs[lane] = rs;
                for (int c = 0; c < P; ++c) sM[lane * LD + c] *= rs;
            }
            __syncthreads();
            if (lane < P) {
                float mx = 0.f;
                for (int r = 0; r < P; ++r) mx = fmaxf(mx, fabsf(sM[r * LD + lane]));
                if (!(mx > 0.f) || !isfinite(mx)) sing = true;
                const float cs = 1.f / mx;
                sCs[lane] = cs;
                for (int r = 0; r < P; ++r) sM[r * LD + lane] *= cs;
            }
            __syncthreads();
            if (__any(sing)) status = LABFM_ST_SINGULAR;

            // ---- FP32 LU with partial pivoting (ties: lowest row)
            int perm = lane;
            if (status == LABFM_ST_OK) {
                for (int kk = 0; kk < P; ++kk) {
                    // pivot: largest |M[r][kk]| over r >= kk, ties to the lowest row
                    const float v = (lane >= kk && lane < P) ? fabsf(sM[lane * LD + kk]) : -1.f;
                    const float vmax = wave_max_float(v);
                    const unsigned long long hit = __ballot(v == vmax);
                    if (!(vmax > 0.f) || !isfinite(vmax) || hit == 0ull) {
                        status = LABFM_ST_SINGULAR;
                        break;
                    }
                    const int pr = __ffsll((long long)hit) - 1;
                    if (pr != kk) {
                        if (lane < P) {
                            const float u = sM[kk * LD + lane];
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
                        const float inv = 1.f / sM[kk * LD + kk];
                        const float u = sM[kk * LD + lane];
                        const bool own = lane == kk;
                        int r = kk + 1;
                        for (; r + 8 <= P; r += 8) {
                            float l[8], a[8];
#pragma unroll
                            for (int e = 0; e < 8; ++e) {
                                l[e] = sM[(r + e) * LD + kk];
                                a[e] = sM[(r + e) * LD + lane];
                            }
#pragma unroll
                            for (int e = 0; e < 8; ++e) {
                                const float m = l[e] * inv;
                                sM[(r + e) * LD + lane] = own ? m : fmaf(-m, u, a[e]);
                            }
                        }
                        for (; r < P; ++r) {
                            const float m = sM[r * LD + kk] * inv;
                            const float a0 = sM[r * LD + lane];
                            sM[r * LD + lane] = own ? m : fmaf(-m, u, a0);
                        }
                    }
                    __syncthreads();
                }
            }
            if (lane < P) sPerm[lane] = perm;
            __syncthreads();

            if (status == LABFM_ST_OK) {
                // ---- Psi from the FP32 factors (or the warm start), weights in FP64
                if (S.psi0 && a.psi0_order == K) {
                    if (lane < P)
                        for (int d = 0; d < nops; ++d)
                            sPsi[d][lane] = (double)S.psi0[i * (int64_t)a.psi0_ld + d * P + lane];
                } else {
                    double b[MAXOPS];
#pragma unroll
                    for (int d = 0; d < MAXOPS; ++d) b[d] = (d < nops && lane < P) ? target(ops.op[d], lane) : 0.0;
                    lu_solve<P, LD, float>(sM, sRs, sCs, sPerm, b, nops);
                    if (lane < P)
#pragma unroll
                        for (int d = 0; d < MAXOPS; ++d)
                            if (d < nops) sPsi[d][lane] = b[d];
                }
                __syncthreads();
                double wreg[JS][MAXOPS];
#pragma unroll
                for (int js = 0; js < JS; ++js) {
                    const int q = lane + 64 * js;
#pragma unroll
                    for (int d = 0; d < MAXOPS; ++d) wreg[js][d] = 0.0;
                    if (q < N) {
                        BasisState<K> B;
                        basis_prepare<K, FAM>(B, dxr[js], dyr[js], a.rbf, a.sigma);
#pragma unroll
                        for (int m = 0; m < P; ++m) {
                            const double wm = abf<K, FAM>(B, m);
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

                // ---- FP64 refinement with FP32 correction solves
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
                    if (!(res > a.tol_stop) || iters >= a.max_iters32) break;
                    lu_solve<P, LD, float>(sM, sRs, sCs, sPerm, r, nops);
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
                            BasisState<K> B;
                            basis_prepare<K, FAM>(B, dxr[js], dyr[js], a.rbf, a.sigma);
                            double dw[MAXOPS];
#pragma unroll
                            for (int d = 0; d < MAXOPS; ++d) dw[d] = 0.0;
#pragma unroll
                            for (int m = 0; m < P; ++m) {
                                const double wm = abf<K, FAM>(B, m);
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
                if (!(res <= a.tol_pass)) {
                    status = LABFM_ST_NOT_CONVERGED;
                } else {
#pragma unroll
                    for (int d = 0; d < MAXOPS; ++d) {
                        if (d >= nops) continue;
                        double hl = 1.0;
                        for (int e = 0; e < deriv_order(ops.op[d]); ++e) hl *= h;
#pragma unroll
                        for (int js = 0; js < JS; ++js) {
                            const int q = lane + 64 * js;
                            if (q < N) {
                                const double wv = wreg[js][d] / hl;
                                if (S.w64) S.w64[(int64_t)d * S.nnz + s0 + q] = wv;
                                if (S.w32) S.w32[(int64_t)d * S.nnz + s0 + q] = (float)wv;
                            }
                        }
                    }
                }
            }
        }
        // nodes the mixed path could not finish (singular FP32 factors or no
        // convergence) are recomputed on the FP64 path; other failures are final
        const bool retry = status == LABFM_ST_NOT_CONVERGED || status == LABFM_ST_SINGULAR;
        if (retry) {
            if (lane == 0) {
                const int pos = atomicAdd(&retry_cnt[K], 1);
                retry_list[list_off[K] + pos] = g;
            }
        } else {
            const bool failed = status != LABFM_ST_OK;
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
                if (S.iters) S.iters[i] = (int8_t)iters;
            }
        }
        __syncthreads();
    }
}

// ---- learned warm start without a factorisation ---------------------------
// Nodes of the network's order take w_j = W(d_j) . Psi0 with the network's
// coefficients as they stand and the FP64 moment residual r = C - X^T w; a
// node at or below tol_pass is finished (iters 0), any other goes to the
// retry list, whose nodes the FP64 LU kernels then solve from scratch.  No
// moment matrix is assembled here.
template <int K, int FAM>
__global__ __launch_bounds__(64) void k_weights_psi0(WeightArgs a, OpList ops, const int32_t* list,
                                                     const int32_t* list_off, const int32_t* list_cnt,
                                                     int32_t* retry_list, int32_t* retry_cnt) {
    constexpr int P = p_of_k(K);
    constexpr int JS = NMAX / 64;
    __shared__ double sD[2][NMAX];
    __shared__ double sWl[MAXOPS][NMAX];
    __shared__ double sPsi[MAXOPS][P];

    const int lane = threadIdx.x;
    const int nops = ops.nops;
    const int count = list_cnt[K];
    const int32_t* mylist = list + list_off[K];

    for (int t = blockIdx.x; t < count; t += gridDim.x) {
        const int32_t g = mylist[t];
        NodeSet S;
        int64_t i;
        resolve(a, g, S, i);
        const int64_t s0 = S.row_ptr[i];
        const int N = (int)(S.row_ptr[i + 1] - s0);
        const double h = 0.5 * S.R[i];
        int status = LABFM_ST_OK;
        double res = INFINITY;

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
                const int q = lane + 64 * js;
                dxr[js] = 0.0;
                dyr[js] = 0.0;
                if (q < N) {
                    const int32_t j = S.col[s0 + q];
                    dxr[js] = min_image(S.x[j] - xi, S.Lx, S.perx) / h;
                    dyr[js] = min_image(S.y[j] - yi, S.Ly, S.pery) / h;
                    sD[0][q] = dxr[js];
                    sD[1][q] = dyr[js];
                    if (FAM != LABFM_ABF_HERMITE && dxr[js] == 0.0 && dyr[js] == 0.0) bad = true;
                }
            }
            if (__any(bad)) status = LABFM_ST_DEGENERATE;
            if (lane < P)
                for (int d = 0; d < nops; ++d) sPsi[d][lane] = (double)S.psi0[i * (int64_t)a.psi0_ld + d * P + lane];
        }
        __syncthreads();

        bool retry = false;
        if (status == LABFM_ST_OK) {
            double wreg[JS][MAXOPS];
#pragma unroll
            for (int js = 0; js < JS; ++js) {
                const int q = lane + 64 * js;
#pragma unroll
                for (int d = 0; d < MAXOPS; ++d) wreg[js][d] = 0.0;
                if (q < N) {
                    BasisState<K> B;
                    basis_prepare<K, FAM>(B, dxr[js], dyr[js], a.rbf, a.sigma);
#pragma unroll
                    for (int m = 0; m < P; ++m) {
                        const double wm = abf<K, FAM>(B, m);
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
            // FP64 moment residual: lane m < P sums over the neighbours
            const int ma = lane < P ? ELEM.a[lane] : 0;
            const int mb = lane < P ? ELEM.b[lane] : 0;
            const double mf = lane < P ? inv_fact(ma) * inv_fact(mb) : 0.0;
            double rm = 0.0;
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
                    if (d < nops) {
                        const double ar = fabs(target(ops.op[d], lane) - accr[d]);
                        rm = (ar > rm || ar != ar) ? ar : rm;
                    }
            }
            if (!isfinite(rm)) rm = INFINITY;
            res = wave_max(rm);
            retry = !(res <= a.tol_pass);
            if (!retry) {
#pragma unroll
                for (int d = 0; d < MAXOPS; ++d) {
                    if (d >= nops) continue;
                    double hl = 1.0;
                    for (int e = 0; e < deriv_order(ops.op[d]); ++e) hl *= h;
#pragma unroll
                    for (int js = 0; js < JS; ++js) {
                        const int q = lane + 64 * js;
                        if (q < N) {
                            const double wv = wreg[js][d] / hl;
                            if (S.w64) S.w64[(int64_t)d * S.nnz + s0 + q] = wv;
                            if (S.w32) S.w32[(int64_t)d * S.nnz + s0 + q] = (float)wv;
                        }
                    }
                }
            }
        }
        if (retry) {
            if (lane == 0) {
                const int pos = atomicAdd(&retry_cnt[K], 1);
                retry_list[list_off[K] + pos] = g;
            }
        } else {
            if (status != LABFM_ST_OK) {
                for (int d = 0; d < nops; ++d)
                    for (int q = lane; q < N; q += 64) {
                        if (S.w64) S.w64[(int64_t)d * S.nnz + s0 + q] = 0.0;
                        if (S.w32) S.w32[(int64_t)d * S.nnz + s0 + q] = 0.0f;
                    }
                res = INFINITY;
            }
            if (lane == 0) {
                S.status[i] = (int8_t)status;
                if (S.resid) S.resid[i] = (float)res;
                if (S.iters) S.iters[i] = 0;
            }
        }
        __syncthreads();
    }
}

template <int K, int FAM>
int grid_for_psi0() {
    static int g = 0;
    if (g == 0) {
        int dev = 0, ncu = 0, per = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_weights_psi0<K, FAM>, 64, 0);
        if (ncu <= 0) ncu = 256;
        if (per <= 0) per = 1;
        g = ncu * per;
    }
    return g;
}

template <int FAM>
void launch_psi0(Context* c, const WeightArgs& a, const OpList& ops, const int32_t* list, const int32_t* off,
                 const int32_t* cnt, int32_t* rlist, int32_t* rcnt, int K, hipStream_t st) {
    KernelTimer timer(c, "weights_psi0", st);
    switch (K) {
        case 1: k_weights_psi0<1, FAM><<<grid_for_psi0<1, FAM>(), 64, 0, st>>>(a, ops, list, off, cnt, rlist, rcnt); break;
        case 2: k_weights_psi0<2, FAM><<<grid_for_psi0<2, FAM>(), 64, 0, st>>>(a, ops, list, off, cnt, rlist, rcnt); break;
        case 3: k_weights_psi0<3, FAM><<<grid_for_psi0<3, FAM>(), 64, 0, st>>>(a, ops, list, off, cnt, rlist, rcnt); break;
        case 4: k_weights_psi0<4, FAM><<<grid_for_psi0<4, FAM>(), 64, 0, st>>>(a, ops, list, off, cnt, rlist, rcnt); break;
        case 5: k_weights_psi0<5, FAM><<<grid_for_psi0<5, FAM>(), 64, 0, st>>>(a, ops, list, off, cnt, rlist, rcnt); break;
        case 6: k_weights_psi0<6, FAM><<<grid_for_psi0<6, FAM>(), 64, 0, st>>>(a, ops, list, off, cnt, rlist, rcnt); break;
        case 7: k_weights_psi0<7, FAM><<<grid_for_psi0<7, FAM>(), 64, 0, st>>>(a, ops, list, off, cnt, rlist, rcnt); break;
        default: k_weights_psi0<8, FAM><<<grid_for_psi0<8, FAM>(), 64, 0, st>>>(a, ops, list, off, cnt, rlist, rcnt); break;
    }
}

template <int K, int FAM>
int grid_for_mixed() {
    static int g = 0;
    if (g == 0) {
        int dev = 0, ncu = 0, per = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_weights_mixed<K, FAM>, 64, 0);
        if (ncu <= 0) ncu = 256;
        if (per <= 0) per = 1;
        g = ncu * per;
    }
    return g;
}

template <int FAM>
void mixed_grids_all() {
    (void)grid_for_mixed<1, FAM>();
    (void)grid_for_mixed<2, FAM>();
    (void)grid_for_mixed<3, FAM>();
    (void)grid_for_mixed<4, FAM>();
    (void)grid_for_mixed<5, FAM>();
    (void)grid_for_mixed<6, FAM>();
    (void)grid_for_mixed<7, FAM>();
    (void)grid_for_mixed<8, FAM>();
}

template <int K, int FAM>
void launch_mixed_one(Context* c, const WeightArgs& a, const OpList& ops, const int32_t* list, const int32_t* off,
                      const int32_t* cnt, int32_t* rlist, int32_t* rcnt, unsigned mask, hipStream_t st) {
    if (!((mask >> K) & 1u)) return;
    static const char* names[KMAX + 1] = {"", "weights32_k1", "weights32_k2", "weights32_k3", "weights32_k4",
                                          "weights32_k5", "weights32_k6", "weights32_k7", "weights32_k8"};
    KernelTimer timer(c, names[K], st);
    k_weights_mixed<K, FAM><<<grid_for_mixed<K, FAM>(), 64, 0, st>>>(a, ops, list, off, cnt, rlist, rcnt);
}

template <int FAM>
void launch_mixed_all(Context* c, const WeightArgs& a, const OpList& ops, const int32_t* list, const int32_t* off,
                      const int32_t* cnt, int32_t* rlist, int32_t* rcnt, unsigned mask, hipStream_t st) {
    launch_mixed_one<1, FAM>(c, a, ops, list, off, cnt, rlist, rcnt, mask, st);
    launch_mixed_one<2, FAM>(c, a, ops, list, off, cnt, rlist, rcnt, mask, st);
    launch_mixed_one<3, FAM>(c, a, ops, list, off, cnt, rlist, rcnt, mask, st);
    launch_mixed_one<4, FAM>(c, a, ops, list, off, cnt, rlist, rcnt, mask, st);
    launch_mixed_one<5, FAM>(c, a, ops, list, off, cnt, rlist, rcnt, mask, st);
    launch_mixed_one<6, FAM>(c, a, ops, list, off, cnt, rlist, rcnt, mask, st);
    launch_mixed_one<7, FAM>(c, a, ops, list, off, cnt, rlist, rcnt, mask, st);
    launch_mixed_one<8, FAM>(c, a, ops, list, off, cnt, rlist, rcnt, mask, st);
}

}  // namespace

void init_mixed_grids() {
    mixed_grids_all<LABFM_ABF_HERMITE>();
    mixed_grids_all<LABFM_ABF_PAPER>();
    mixed_grids_all<LABFM_ABF_PAPER_D1>();
}

// Mixed kernels of the orders in `mask` over given lists, then FP64 kernels on
// the nodes they hand back.  rl: >= ntotal + KMAX + 2 int32 (counters first).
labfm_err weights_mixed_lists(Context* c, const WeightArgs& a0, const int32_t* list, const int32_t* off,
                              const int32_t* cnt, int32_t* rl, unsigned mask, hipStream_t st, int direct_order,
                              Scratch* fp64_ws) {
    int32_t* rcnt = rl;
    int32_t* rlist = rcnt + (KMAX + 2);
    labfm_err e = fill_i32(rcnt, KMAX + 2, 0, st);
    if (e != LABFM_OK) return e;
    OpList ops{};
    ops.nops = 0;
    for (int b = 0; b < 5; ++b)
        if (a0.ops & (1u << b)) ops.op[ops.nops++] = 1u << b;
    unsigned mixed_mask = mask;
    if (direct_order >= 1 && direct_order <= KMAX && ((mask >> direct_order) & 1u)) {
        mixed_mask &= ~(1u << direct_order);
        if (a0.abf == LABFM_ABF_HERMITE)
            launch_psi0<LABFM_ABF_HERMITE>(c, a0, ops, list, off, cnt, rlist, rcnt, direct_order, st);
        else if (a0.abf == LABFM_ABF_PAPER)
            launch_psi0<LABFM_ABF_PAPER>(c, a0, ops, list, off, cnt, rlist, rcnt, direct_order, st);
        else
            launch_psi0<LABFM_ABF_PAPER_D1>(c, a0, ops, list, off, cnt, rlist, rcnt, direct_order, st);
    }
    if (a0.abf == LABFM_ABF_HERMITE)
        launch_mixed_all<LABFM_ABF_HERMITE>(c, a0, ops, list, off, cnt, rlist, rcnt, mixed_mask, st);
    else if (a0.abf == LABFM_ABF_PAPER)
        launch_mixed_all<LABFM_ABF_PAPER>(c, a0, ops, list, off, cnt, rlist, rcnt, mixed_mask, st);
    else
        launch_mixed_all<LABFM_ABF_PAPER_D1>(c, a0, ops, list, off, cnt, rlist, rcnt, mixed_mask, st);
    LABFM_HIP_CHECK(hipGetLastError());
    // FP64 recomputation of the retry list; iters of those nodes are offset by 64
    WeightArgs a = a0;
    a.iters_offset = 64;
    if (fp64_ws) return weights_fp64_split_lists(c, a, rlist, off, rcnt, mask, *fp64_ws, st);
    return weights_fp64_lists(c, a, rlist, off, rcnt, mask, st);
}

labfm_err weights_mixed(Context* c, const WeightArgs& a0, const NodeSet* hs, int32_t* wl, int32_t* rl,
                        unsigned fp64_orders, hipStream_t st, int direct_order, Scratch* fp64_ws) {
    int32_t *list = wl, *off, *cnt;
    labfm_err e = build_order_lists(c, a0, hs, st, &list, &off, &cnt);
    if (e != LABFM_OK) return e;
    if ((e = weights_invalid_orders(a0, list, off, cnt, st)) != LABFM_OK) return e;
    if (fp64_orders & ALL_ORDERS) {
        e = fp64_ws ? weights_fp64_split_lists(c, a0, list, off, cnt, fp64_orders & ALL_ORDERS, *fp64_ws, st)
                    : weights_fp64_lists(c, a0, list, off, cnt, fp64_orders & ALL_ORDERS, st);
        if (e != LABFM_OK) return e;
    }
    return weights_mixed_lists(c, a0, list, off, cnt, rl, ALL_ORDERS & ~fp64_orders, st, direct_order, fp64_ws);
}

}  // namespace labfm
