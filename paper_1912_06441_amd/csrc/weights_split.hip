// weights_split.hip -- per-node LABFM weights on gfx950, FP64, in two kernels.
//
// The same computation as the single FP64 kernel (Sec. 3.1 of King, Lind &
// Nasar: M = sum_j X(d_j) W(d_j)^T, M Psi = C, w = W Psi, refinement on the
// moment residual r = C - X^T w), split where its resource needs change:
//   * k_factor64: assembly, equilibration, partial-pivot LU and the first
//     solve.  The basis chunks share M's LDS buffer (they are read only while
//     M is still in registers), so two node systems run per SIMD.  The LU
//     keeps one row of M per lane in registers and pivots by place instead of
//     moving rows: each elimination step broadcasts the pivot row by
//     readlane (four entries at a time, in uniform control flow) and only the
//     rows below the pivot take the update, without touching LDS.
//   * k_refine64: weights w = W Psi, the FP64 moment residual and the
//     refinement.  A node that needs a correction reads its factors back
//     straight into registers (lane r takes row r), so the kernel keeps no
//     P x P matrix in LDS and two node systems run per SIMD.
// Between the two, per node of the current chunk of a work list: the LU
// factors (P x P, column-major), row and column scales, the row at each
// pivot place, Psi and the status, in a workspace of FACTOR_SLOTS node slots.  Every step and
// every rounding is the single kernel's, so the results are the same.
#include "weights_common.hpp"

namespace labfm {

namespace {
using namespace wk;

struct FactorWs {
    double* lu;     // [slots][P * P], column-major: entry (r, c) at c * P + r
    double* rs;     // [slots][P]
    double* cs;     // [slots][P]
    double* psi;    // [slots][MAXOPS][P]
    int32_t* perm;  // [slots][P]: the row (of the equilibrated M) at each place
    int8_t* st;     // [slots]
};

// Operator slots 0..NB-1 are always computed: a call with fewer operators
// runs them on zero coefficients (zero right-hand sides, so zero solutions),
// which keeps the common three-operator case free of per-slot branches.
// Slots beyond NB follow the run-time count.
constexpr int NB = 3;
__device__ inline bool live(int d, int nops) { return d < NB || d < nops; }

// v of another lane of the same row of 16, by a DPP move of both halves
// (CTRL 0x121..0x12f: rotate the row right by 1..15 lanes)
template <int CTRL>
__device__ inline double dpp_d(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// Maximum over the wavefront: rotations by 8, 4, 2 and 1 lanes leave every
// lane with its row's maximum, then the four row maxima are combined.  fmax
// skips NaN in any order, so the result is the same as a butterfly's.
__device__ inline double wave_max_dpp(double v) {
    v = fmax(v, dpp_d<0x128>(v));
    v = fmax(v, dpp_d<0x124>(v));
    v = fmax(v, dpp_d<0x122>(v));
    v = fmax(v, dpp_d<0x121>(v));
    return fmax(fmax(bcast(v, 0), bcast(v, 16)), fmax(bcast(v, 32), bcast(v, 48)));
}

template <int K, int FAM>
__global__ __launch_bounds__(64) void k_factor64(WeightArgs a, OpList ops, const int32_t* list,
                                                 const int32_t* list_off, const int32_t* list_cnt, int begin, int end,
                                                 FactorWs w) {
    constexpr int P = p_of_k(K);
    constexpr int BS = (P + 7) / 8;
    constexpr int PP = 8 * BS;
    constexpr int LD = P + 1;
    constexpr int JS = NMAX / 64;

    // M and the basis chunks share one buffer: the chunks are read only during
    // the assembly, which keeps M in registers and writes it after the last
    // chunk's barrier.
    __shared__ double sMC[cmax(P * LD, 2 * CH * PP)];
    double* const sM = sMC;
    double* const sChunk = sMC;  // basis chunk: X then W
    __shared__ double sD[2][NMAX];
    __shared__ double sRs[P], sCs[P];
    __shared__ int sPerm[P];

    const int lane = threadIdx.x;
    const int nops = ops.nops;
    const int count = min(list_cnt[K], end);
    const int32_t* mylist = list + list_off[K];

    for (int t = begin + blockIdx.x; t < count; t += gridDim.x) {
        const int64_t slot = t - begin;
        NodeSet S;
        int64_t i;
        resolve(a, mylist[t], S, i);
        const int64_t s0 = S.row_ptr[i];
        const int N = (int)(S.row_ptr[i + 1] - s0);
        const double h = 0.5 * S.R[i];
        int status = LABFM_ST_OK;

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

            // ---- LU with partial pivoting, one row per lane in registers.  Rows
            // stay in the lanes they were assembled in; pos is a row's place in
            // the pivoted order, and ties of the pivot search go to the lowest
            // place, as when rows are swapped in memory.
            double row[P];
#pragma unroll
            for (int c = 0; c < P; ++c) row[c] = lane < P ? sM[lane * LD + c] : 0.0;
            int pos = lane;  // lanes >= P are never candidates and never updated
            if (status == LABFM_ST_OK) {
#pragma unroll
                for (int kk = 0; kk < P; ++kk) {
                    const double v = (pos >= kk && pos < P) ? fabs(row[kk]) : -1.0;
                    const double vmax = wave_max_dpp(v);
                    const unsigned long long hit = __ballot(v == vmax);
                    if (!(vmax > 0.0) || !isfinite(vmax) || hit == 0ull) {
                        status = LABFM_ST_SINGULAR;
                        break;
                    }
                    int pl = __ffsll((long long)hit) - 1;
                    if (__popcll(hit) > 1) {  // tied candidates: the lowest place wins
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
                    // pivot-row entries are read in uniform control flow, a group at a
                    // time; only the rows below the pivot take the update
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
            if (lane < P) sPerm[pos] = lane;  // place -> row
            __syncthreads();
            if (status == LABFM_ST_OK) {
                // ---- initial solve: lane m holds C^d[m] for row m; the value of
                // place c lives in lane sPerm[c]
                double t[MAXOPS];
                const double rs = lane < P ? sRs[lane] : 0.0;
#pragma unroll
                for (int d = 0; d < MAXOPS; ++d) t[d] = ((d < nops) ? target(ops.op[d], lane) : 0.0) * rs;
                const int perm_reg = lane < P ? sPerm[lane] : 0;  // lane c: the row at place c
#pragma unroll
                for (int c = 0; c < P - 1; ++c) {
                    const int src = __builtin_amdgcn_readlane(perm_reg, c);
                    const double l = (pos > c && pos < P) ? row[c] : 0.0;
#pragma unroll
                    for (int d = 0; d < MAXOPS; ++d)
                        if (live(d, nops)) t[d] -= l * bcast(t[d], src);
                }
#pragma unroll
                for (int c = P - 1; c >= 0; --c) {
                    const int src = __builtin_amdgcn_readlane(perm_reg, c);
                    const double u = pos < c ? row[c] : 0.0;
#pragma unroll
                    for (int d = 0; d < MAXOPS; ++d) {
                        if (live(d, nops)) {
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

// Solve M z = b with the equilibrated, pivoted LU of one node read from the
// workspace: lane r loads row r of the factors (column c of the stored
// column-major matrix is one contiguous load across the lanes), so the solve
// runs in registers.  The arithmetic, and its order, is lu_solve's.
template <int P>
__device__ inline void lu_solve_rows(const double* lu_node, double rs, double cs, int pr, double (&b)[MAXOPS],
                                     int nops) {
    const int lane = threadIdx.x;
    // The base pointer passes through an empty asm so that the compiler forms
    // the column addresses here, at each call, instead of hoisting all P of
    // them out of the refinement loop into scalar registers (which then spill).
    uint64_t bits = (uint64_t)lu_node;
    asm volatile("" : "+s"(bits));
    const double* lu = (const double*)bits;
    double t[MAXOPS];
#pragma unroll
    for (int d = 0; d < MAXOPS; ++d) {
        double v = b[d] * rs;
        t[d] = __shfl(v, pr, 64);
    }
    // the whole row at once: the lower part for the forward pass, the upper
    // part and the diagonal for the backward pass
    double row[P];
#pragma unroll
    for (int c = 0; c < P; ++c) row[c] = lane < P ? lu[c * P + lane] : 0.0;
    // forward: unit lower triangle
#pragma unroll
    for (int c = 0; c < P - 1; ++c) {
        const double l = lane > c ? row[c] : 0.0;
#pragma unroll
        for (int d = 0; d < MAXOPS; ++d)
            if (live(d, nops)) t[d] -= l * bcast(t[d], c);
    }
    // backward: lane c divides by its diagonal, lanes above it subtract
#pragma unroll
    for (int c = P - 1; c >= 0; --c) {
        const double u = lane < c ? row[c] : 0.0;
#pragma unroll
        for (int d = 0; d < MAXOPS; ++d) {
            if (live(d, nops)) {
                const double q = t[d] / row[c];  // every lane divides; lane c keeps it
                t[d] = lane == c ? q : t[d];
                t[d] -= u * bcast(t[d], c);
            }
        }
    }
#pragma unroll
    for (int d = 0; d < MAXOPS; ++d) b[d] = t[d] * cs;
}

template <int K, int FAM>
__global__ __launch_bounds__(64) void k_refine64(WeightArgs a, OpList ops, const int32_t* list,
                                                 const int32_t* list_off, const int32_t* list_cnt, int begin, int end,
                                                 FactorWs w) {
    constexpr int P = p_of_k(K);
    constexpr int BS = (P + 7) / 8;
    constexpr int PP = 8 * BS;

    __shared__ double sD[2][NMAX];
    __shared__ double sWl[MAXOPS][NMAX];    // scaled weights: the running sums, and the residual's input
    __shared__ double sPsi[MAXOPS][PP];     // solution / correction coefficients

    const int lane = threadIdx.x;
    const int nops = ops.nops;
    const int count = min(list_cnt[K], end);
    const int32_t* mylist = list + list_off[K];

    for (int t = begin + blockIdx.x; t < count; t += gridDim.x) {
        const int64_t slot = t - begin;
        NodeSet S;
        int64_t i;
        resolve(a, mylist[t], S, i);
        const int64_t s0 = S.row_ptr[i];
        const int N = (int)(S.row_ptr[i + 1] - s0);
        const double h = 0.5 * S.R[i];
        int status = w.st[slot];
        double res = INFINITY;
        int iters = 0;

        if (status == LABFM_ST_OK) {
            const double xi = S.x[i], yi = S.y[i];
            for (int q = lane; q < N; q += 64) {
                int32_t j = S.col[s0 + q];
                sD[0][q] = min_image(S.x[j] - xi, S.Lx, S.perx) / h;
                sD[1][q] = min_image(S.y[j] - yi, S.Ly, S.pery) / h;
            }
            if (lane < P)
                for (int d = 0; d < MAXOPS; ++d)
                    if (live(d, nops)) sPsi[d][lane] = d < nops ? w.psi[(slot * MAXOPS + d) * (int64_t)P + lane] : 0.0;
        }
        __syncthreads();

        if (status == LABFM_ST_OK) {
            {
                // ---- w_j = W(d_j) . Psi (lane q keeps neighbour q's sums in sWl)
                for (int q = lane; q < N; q += 64) {
                    asm volatile("" ::: "memory");  // keeps Psi's loads inside the loop (not held in registers)
                    double wv[MAXOPS];
#pragma unroll
                    for (int d = 0; d < MAXOPS; ++d) wv[d] = 0.0;
                    BasisState<K> B;
                    basis_prepare<K, FAM>(B, sD[0][q], sD[1][q], a.rbf, a.sigma);
#pragma unroll
                    for (int m = 0; m < P; ++m) {
                        double wm = abf<K, FAM>(B, m);
#pragma unroll
                        for (int d = 0; d < MAXOPS; ++d)
                            if (live(d, nops)) wv[d] = fma(wm, sPsi[d][m], wv[d]);
                    }
#pragma unroll
                    for (int d = 0; d < MAXOPS; ++d)
                        if (live(d, nops)) sWl[d][q] = wv[d];
                }
                __syncthreads();

                // the factors of this node, loaded by lane m on the first correction
                const double* lu = w.lu + slot * (int64_t)(P * P);
                double rs = 0.0, cs = 0.0;
                int pr = 0;
                bool lu_in = false;

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
                        // every slot's sum is read and accumulated without a branch (a slot
                        // beyond the operator count holds values that are never used), and four
                        // neighbours are loaded ahead, so the LDS reads overlap
#pragma unroll 4
                        for (int q = 0; q < N; ++q) {
                            const double dx = sD[0][q], dy = sD[1][q];
                            double wv[MAXOPS];
#pragma unroll
                            for (int d = 0; d < MAXOPS; ++d) wv[d] = sWl[d][q];
                            double xm = mf;
#pragma unroll
                            for (int e = 0; e < K; ++e) {
                                xm *= (e < ma) ? dx : 1.0;
                                xm *= (e < mb) ? dy : 1.0;
                            }
#pragma unroll
                            for (int d = 0; d < MAXOPS; ++d) accr[d] = fma(xm, wv[d], accr[d]);
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
                    if (!lu_in) {
                        if (lane < P) {
                            rs = w.rs[slot * (int64_t)P + lane];
                            cs = w.cs[slot * (int64_t)P + lane];
                            pr = w.perm[slot * (int64_t)P + lane];
                        }
                        lu_in = true;
                    }
                    lu_solve_rows<P>(lu, rs, cs, pr, r, nops);
                    if (lane < P)
#pragma unroll
                        for (int d = 0; d < MAXOPS; ++d)
                            if (live(d, nops)) sPsi[d][lane] = r[d];
                    __syncthreads();
                    for (int q = lane; q < N; q += 64) {
                        asm volatile("" ::: "memory");  // as above
                        BasisState<K> B;
                        basis_prepare<K, FAM>(B, sD[0][q], sD[1][q], a.rbf, a.sigma);
                        double dw[MAXOPS];
#pragma unroll
                        for (int d = 0; d < MAXOPS; ++d) dw[d] = 0.0;
#pragma unroll
                        for (int m = 0; m < P; ++m) {
                            double wm = abf<K, FAM>(B, m);
#pragma unroll
                            for (int d = 0; d < MAXOPS; ++d)
                                if (live(d, nops)) dw[d] = fma(wm, sPsi[d][m], dw[d]);
                        }
#pragma unroll
                        for (int d = 0; d < MAXOPS; ++d)
                            if (live(d, nops)) sWl[d][q] += dw[d];
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
                    for (int q = lane; q < N; q += 64) {
                        double wv = sWl[d][q] / hl;
                        if (S.w64) S.w64[(int64_t)d * S.nnz + s0 + q] = wv;
                        if (S.w32) S.w32[(int64_t)d * S.nnz + s0 + q] = (float)wv;
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

template <typename Kern>
int split_grid(Kern kern) {
    int dev = 0, ncu = 0, per = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, 64, 0);
    if (ncu <= 0) ncu = 256;
    if (per <= 0) per = 1;
    return ncu * per;
}

// persistent grid sizes (workgroups resident at once), set before the first launch
template <int K, int FAM>
int& grid_factor() {
    static int g = 0;
    return g;
}
template <int K, int FAM>
int& grid_refine() {
    static int g = 0;
    return g;
}
template <int K, int FAM>
void init_grid() {
    if (grid_factor<K, FAM>() == 0) grid_factor<K, FAM>() = split_grid(k_factor64<K, FAM>);
    if (grid_refine<K, FAM>() == 0) grid_refine<K, FAM>() = split_grid(k_refine64<K, FAM>);
}
template <int FAM>
void init_grids() {
    init_grid<1, FAM>();
    init_grid<2, FAM>();
    init_grid<3, FAM>();
    init_grid<4, FAM>();
    init_grid<5, FAM>();
    init_grid<6, FAM>();
    init_grid<7, FAM>();
    init_grid<8, FAM>();
}

template <int K, int FAM>
void launch_split(Context* c, const WeightArgs& a, const OpList& ops, const int32_t* list, const int32_t* off,
                  const int32_t* cnt, unsigned mask, int begin, int end, const FactorWs& w, hipStream_t st) {
    if (!((mask >> K) & 1u)) return;
    init_grid<K, FAM>();
    static const char* fnames[KMAX + 1] = {"",              "weights64f_k1", "weights64f_k2", "weights64f_k3",
                                           "weights64f_k4", "weights64f_k5", "weights64f_k6", "weights64f_k7",
                                           "weights64f_k8"};
    static const char* rnames[KMAX + 1] = {"",              "weights64r_k1", "weights64r_k2", "weights64r_k3",
                                           "weights64r_k4", "weights64r_k5", "weights64r_k6", "weights64r_k7",
                                           "weights64r_k8"};
    {
        KernelTimer timer(c, fnames[K], st);
        k_factor64<K, FAM><<<grid_factor<K, FAM>(), 64, 0, st>>>(a, ops, list, off, cnt, begin, end, w);
    }
    {
        KernelTimer timer(c, rnames[K], st);
        k_refine64<K, FAM><<<grid_refine<K, FAM>(), 64, 0, st>>>(a, ops, list, off, cnt, begin, end, w);
    }
}

template <int FAM>
void launch_split_all(Context* c, const WeightArgs& a, const OpList& ops, const int32_t* list, const int32_t* off,
                      const int32_t* cnt, unsigned mask, int begin, int end, const FactorWs& w, hipStream_t st) {
    launch_split<1, FAM>(c, a, ops, list, off, cnt, mask, begin, end, w, st);
    launch_split<2, FAM>(c, a, ops, list, off, cnt, mask, begin, end, w, st);
    launch_split<3, FAM>(c, a, ops, list, off, cnt, mask, begin, end, w, st);
    launch_split<4, FAM>(c, a, ops, list, off, cnt, mask, begin, end, w, st);
    launch_split<5, FAM>(c, a, ops, list, off, cnt, mask, begin, end, w, st);
    launch_split<6, FAM>(c, a, ops, list, off, cnt, mask, begin, end, w, st);
    launch_split<7, FAM>(c, a, ops, list, off, cnt, mask, begin, end, w, st);
    launch_split<8, FAM>(c, a, ops, list, off, cnt, mask, begin, end, w, st);
}

// Node slots of the workspace: one chunk of a work list at a time (about
// 4.8 GB at order 8); larger calls take several chunks.
constexpr int64_t FACTOR_SLOTS = 1 << 18;

int64_t slots_for(int64_t ntotal) { return ntotal < FACTOR_SLOTS ? (ntotal > 0 ? ntotal : 1) : FACTOR_SLOTS; }

// workspace layout for `slots` node slots, each sized for the largest order
FactorWs carve(void* p, int64_t slots) {
    constexpr int64_t PM = p_of_k(KMAX);
    const size_t b_lu = sizeof(double) * (size_t)(slots * PM * PM);
    const size_t b_sc = sizeof(double) * (size_t)(slots * PM);
    const size_t b_psi = sizeof(double) * (size_t)(slots * MAXOPS * PM);
    const size_t b_perm = sizeof(int32_t) * (size_t)(slots * PM);
    char* base = (char*)p;
    FactorWs w;
    w.lu = (double*)base;
    w.rs = (double*)(base + b_lu);
    w.cs = (double*)(base + b_lu + b_sc);
    w.psi = (double*)(base + b_lu + 2 * b_sc);
    w.perm = (int32_t*)(base + b_lu + 2 * b_sc + b_psi);
    w.st = (int8_t*)(base + b_lu + 2 * b_sc + b_psi + b_perm);
    return w;
}

size_t workspace_bytes(int64_t slots) {
    constexpr int64_t PM = p_of_k(KMAX);
    return sizeof(double) * (size_t)(slots * PM * PM) + 2 * sizeof(double) * (size_t)(slots * PM) +
           sizeof(double) * (size_t)(slots * MAXOPS * PM) + sizeof(int32_t) * (size_t)(slots * PM) + (size_t)slots;
}

}  // namespace

void init_split_grids() {
    init_grids<LABFM_ABF_HERMITE>();
    init_grids<LABFM_ABF_PAPER>();
    init_grids<LABFM_ABF_PAPER_D1>();
}

labfm_err fp64_split_reserve(Scratch& ws, int64_t ntotal) { return ensure(ws, workspace_bytes(slots_for(ntotal))); }

labfm_err weights_fp64_split_lists(Context* c, const WeightArgs& a, const int32_t* list, const int32_t* off,
                                   const int32_t* cnt, unsigned mask, Scratch& ws, hipStream_t st) {
    const int64_t slots = slots_for(a.ntotal);
    labfm_err e = ensure(ws, workspace_bytes(slots));
    if (e != LABFM_OK) return e;
    const FactorWs w = carve(ws.p, slots);
    OpList ops{};
    ops.nops = 0;
    for (int b = 0; b < 5; ++b)
        if (a.ops & (1u << b)) ops.op[ops.nops++] = 1u << b;
    for (int64_t b0 = 0; b0 < a.ntotal; b0 += slots) {
        const int begin = (int)b0;
        const int end = (int)(b0 + slots < a.ntotal ? b0 + slots : a.ntotal);
        if (a.abf == LABFM_ABF_HERMITE)
            launch_split_all<LABFM_ABF_HERMITE>(c, a, ops, list, off, cnt, mask, begin, end, w, st);
        else if (a.abf == LABFM_ABF_PAPER)
            launch_split_all<LABFM_ABF_PAPER>(c, a, ops, list, off, cnt, mask, begin, end, w, st);
        else
            launch_split_all<LABFM_ABF_PAPER_D1>(c, a, ops, list, off, cnt, mask, begin, end, w, st);
        LABFM_HIP_CHECK(hipGetLastError());
    }
    return LABFM_OK;
}

labfm_err weights_fp64_split(Context* c, const WeightArgs& a, const NodeSet* hs, int32_t* wl, Scratch& ws,
                             hipStream_t st) {
    int32_t *list = wl, *off, *cnt;
    labfm_err e = build_order_lists(c, a, hs, st, &list, &off, &cnt);
    if (e != LABFM_OK) return e;
    if ((e = weights_invalid_orders(a, list, off, cnt, st)) != LABFM_OK) return e;
    return weights_fp64_split_lists(c, a, list, off, cnt, ALL_ORDERS, ws, st);
}

}  // namespace labfm
