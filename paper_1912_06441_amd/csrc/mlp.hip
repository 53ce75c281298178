// mlp.hip -- learned warm start for the per-node weight solve.
//
// A fully connected network maps the scaled offsets of a stencil's nearest
// neighbours to the ABF coefficients Psi^d of the moment system M Psi = C
// (Sec. 3.1 eq. lsys of King, Lind & Nasar); the FP64 weight refinement of
// the mixed path then starts from W Psi instead of from a first solve.
// Kernels here:
//   * k_features: per node, neighbours ranked by (squared scaled distance,
//     index) in one wavefront; the nearest kmax written as (dx/h, dy/h, 1).
//   * k_gemm: C = epi(A B) on the matrix cores (v_mfma_f32_16x16x32_bf16:
//     BF16 operands, FP32 accumulation), 64x64 tiles staged through LDS; the
//     epilogue adds the bias and applies SiLU, the output de-normalisation or
//     the SiLU derivative, so every layer of forward and backward is one GEMM.
//   * column sums for the bias gradients, the moment-residual loss and its
//     gradient, Adam, and the FP32 -> BF16 cast of the parameters.
//
// MFMA lane layout (16x16x32, wave64): lane l holds A[l%16][8(l/16)..8(l/16)+7]
// and B[8(l/16)..8(l/16)+7][l%16]; result register i of lane l is row
// 4(l/16)+i, column l%16.  Both LDS tiles are stored K-contiguous so each
// operand is one 16-byte LDS read.
#include <cmath>

#include "weights_common.hpp"

namespace labfm {

namespace {
using namespace wk;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// Logistic function 1 / (1 + e^-z) = 1 / (1 + 2^(-z log2 e)) from the
// hardware base-2 exponential and reciprocal (about one ulp each in FP32).
// The activations it produces are rounded to BF16 (8-bit significand) or
// enter FP32 gradients of a BF16 network, so the IEEE-rounded exp and divide
// buy nothing here.  Large |z| saturate correctly: 2^+inf = inf -> 0, 2^-inf = 0 -> 1.
__device__ inline float logistic(float z) {
    return __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(z * -1.44269504088896341f));
}

// ------------------------------------------------------------------ features

__global__ __launch_bounds__(64) void k_features(const double* __restrict__ x, const double* __restrict__ y,
                                                 const double* __restrict__ R, const int64_t* __restrict__ rp,
                                                 const int32_t* __restrict__ col, int64_t first, int64_t count,
                                                 double Lx, double Ly, int perx, int pery, int kmax,
                                                 float* __restrict__ feat) {
    __shared__ double sd2[NMAX];
    const int lane = threadIdx.x;
    for (int64_t t = blockIdx.x; t < count; t += gridDim.x) {
        const int64_t i = first + t;
        const int64_t s0 = rp[i];
        const int N = (int)(rp[i + 1] - s0);
        float* out = feat + t * (int64_t)(3 * kmax);
        if (N > NMAX) {  // not an admissible stencil: no features
            for (int q = lane; q < 3 * kmax; q += 64) out[q] = 0.f;
            continue;
        }
        const double xi = x[i], yi = y[i], h = 0.5 * R[i];
        double dxv[NMAX / 64], dyv[NMAX / 64], d2v[NMAX / 64];
#pragma unroll
        for (int js = 0; js < NMAX / 64; ++js) {
            const int q = lane + 64 * js;
            dxv[js] = dyv[js] = d2v[js] = 0.0;
            if (q < N) {
                const int32_t j = col[s0 + q];
                dxv[js] = min_image(x[j] - xi, Lx, perx) / h;
                dyv[js] = min_image(y[j] - yi, Ly, pery) / h;
                // no contraction: the ranking must see exactly dx*dx + dy*dy
                d2v[js] = __dadd_rn(__dmul_rn(dxv[js], dxv[js]), __dmul_rn(dyv[js], dyv[js]));
                sd2[q] = d2v[js];
            }
        }
        __syncthreads();
#pragma unroll
        for (int js = 0; js < NMAX / 64; ++js) {
            const int q = lane + 64 * js;
            if (q < N) {
                int rank = 0;
                for (int q2 = 0; q2 < N; ++q2) {
                    const double e = sd2[q2];
                    rank += (e < d2v[js]) || (e == d2v[js] && q2 < q);
                }
                if (rank < kmax) {
                    out[3 * rank] = (float)dxv[js];
                    out[3 * rank + 1] = (float)dyv[js];
                    out[3 * rank + 2] = 1.f;
                }
            }
        }
        const int kv = N < kmax ? N : kmax;
        for (int q = 3 * kv + lane; q < 3 * kmax; q += 64) out[q] = 0.f;
        __syncthreads();
    }
}

// ------------------------------------------------------------------ GEMM

constexpr int GBM = 64, GBN = 64, GBK = 32, GLD = GBK + 8;
enum { EPI_PLAIN = 0, EPI_SILU = 1, EPI_LINEAR = 2, EPI_DSILU = 3 };

struct GemmArgs {
    int M, N, K;
    const float* A;  // element (m, k) at A[m * lam + k * lak]
    int64_t lam, lak;
    const void* B;   // element (k, n) at B[k * lbk + n * lbn]
    int64_t lbk, lbn;
    float* C;        // element (m, n) at C[m * ldc + n]
    int64_t ldc;
    const float* bias;  // [N] (SILU, LINEAR; may be NULL for LINEAR)
    const float* mu;    // [N] output shift (LINEAR, optional)
    const float* sd;    // [N] output scale (LINEAR, with mu)
    float* zout;        // pre-activations (SILU, optional), same layout as C
    const float* zin;   // pre-activations (DSILU), same layout as C
};

__device__ inline float to_f(float v) { return v; }
__device__ inline float to_f(__bf16 v) { return (float)v; }

// AK: A contiguous along k (lak == 1), else along m (lam == 1); BK likewise.
template <typename TB, bool AK, bool BK, int EPI>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
    __shared__ __bf16 As[GBM][GLD];
    __shared__ __bf16 Bs[GBN][GLD];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int m0 = blockIdx.y * GBM, n0 = blockIdx.x * GBN;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    const TB* B = (const TB*)g.B;
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < g.K; k0 += GBK) {
        if (AK) {
            const int m = tid >> 2, kq = (tid & 3) * 8, gm = m0 + m;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int gk = k0 + kq + e;
                const float v = (gm < g.M && gk < g.K) ? g.A[(int64_t)gm * g.lam + gk] : 0.f;
                As[m][kq + e] = (__bf16)v;
            }
        } else {
            const int k = tid >> 3, mq = (tid & 7) * 8, gk = k0 + k;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int gm = m0 + mq + e;
                const float v = (gm < g.M && gk < g.K) ? g.A[gm + (int64_t)gk * g.lak] : 0.f;
                As[mq + e][k] = (__bf16)v;
            }
        }
        if (BK) {
            const int n = tid >> 2, kq = (tid & 3) * 8, gn = n0 + n;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int gk = k0 + kq + e;
                const float v = (gn < g.N && gk < g.K) ? to_f(B[(int64_t)gn * g.lbn + gk]) : 0.f;
                Bs[n][kq + e] = (__bf16)v;
            }
        } else {
            const int k = tid >> 3, nq = (tid & 7) * 8, gk = k0 + k;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int gn = n0 + nq + e;
                const float v = (gn < g.N && gk < g.K) ? to_f(B[(int64_t)gk * g.lbk + gn]) : 0.f;
                Bs[nq + e][k] = (__bf16)v;
            }
        }
        __syncthreads();
        bf16x8 af[2], bf[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) af[i] = *(const bf16x8*)&As[wm + 16 * i + (lane & 15)][8 * (lane >> 4)];
#pragma unroll
        for (int j = 0; j < 2; ++j) bf[j] = *(const bf16x8*)&Bs[wn + 16 * j + (lane & 15)][8 * (lane >> 4)];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }

#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
                const int cn = n0 + wn + 16 * j + (lane & 15);
                if (row >= g.M || cn >= g.N) continue;
                const float v = acc[i][j][r];
                const int64_t o = (int64_t)row * g.ldc + cn;
                if (EPI == EPI_PLAIN) {
                    g.C[o] = v;
                } else if (EPI == EPI_SILU) {
                    const float z = v + g.bias[cn];
                    if (g.zout) g.zout[o] = z;
                    g.C[o] = z * logistic(z);
                } else if (EPI == EPI_LINEAR) {
                    float z = v + (g.bias ? g.bias[cn] : 0.f);
                    if (g.mu) z = g.mu[cn] + g.sd[cn] * z;
                    g.C[o] = z;
                } else {
                    const float z = g.zin[o];
                    const float s = logistic(z);
                    g.C[o] = v * s * (1.f + z * (1.f - s));
                }
            }
}

// Forward layers (A FP32 [M][K] row-major, W BF16 [N][K] row-major, K a
// multiple of 32, 16-byte aligned rows): 128 x 128 block tiles, each of the
// four waves computes 64 x 64 (4 x 4 MFMA tiles); A and W tiles are loaded
// 16 bytes per access and double-buffered in LDS, one barrier per k-step.
constexpr int FBM = 128, FBN = 128, FBK = 32, FLD = FBK + 8;

template <int EPI>
__global__ __launch_bounds__(256) void k_gemm_fwd(GemmArgs g) {
    __shared__ __bf16 As[2][FBM][FLD];
    __shared__ __bf16 Bs[2][FBN][FLD];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int m0 = blockIdx.y * FBM, n0 = blockIdx.x * FBN;
    const int wm = (w >> 1) * 64, wn = (w & 1) * 64;
    const __bf16* W = (const __bf16*)g.B;
    // loader: thread t covers row t/2, 16 consecutive k at (t%2)*16
    const int lr = tid >> 1, lk = (tid & 1) * 16;
    const int gm = m0 + lr, gn = n0 + lr;
    const bool am = gm < g.M, bn = gn < g.N;
    const float* arow = g.A + (int64_t)(am ? gm : 0) * g.lam + lk;
    const __bf16* brow = W + (int64_t)(bn ? gn : 0) * g.lbn + lk;
    floatx4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    floatx4 ra[4];
    bf16x8 rb[2];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) ra[q] = am ? *(const floatx4*)(arow + k0 + 4 * q) : floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            if (bn) {
                rb[q] = *(const bf16x8*)(brow + k0 + 8 * q);
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) rb[q][e] = (__bf16)0.f;
            }
        }
    };
    auto stash = [&](int buf) {
        bf16x8 a0, a1;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            a0[e] = (__bf16)ra[0][e];
            a0[4 + e] = (__bf16)ra[1][e];
            a1[e] = (__bf16)ra[2][e];
            a1[4 + e] = (__bf16)ra[3][e];
        }
        *(bf16x8*)&As[buf][lr][lk] = a0;
        *(bf16x8*)&As[buf][lr][lk + 8] = a1;
        *(bf16x8*)&Bs[buf][lr][lk] = rb[0];
        *(bf16x8*)&Bs[buf][lr][lk + 8] = rb[1];
    };
    const int nk = g.K / FBK;
    load(0);
    stash(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) load((kt + 1) * FBK);  // next tile in flight during the products
        bf16x8 af[4], bf[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) af[i] = *(const bf16x8*)&As[cur][wm + 16 * i + (lane & 15)][8 * (lane >> 4)];
#pragma unroll
        for (int j = 0; j < 4; ++j) bf[j] = *(const bf16x8*)&Bs[cur][wn + 16 * j + (lane & 15)][8 * (lane >> 4)];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
        if (kt + 1 < nk) stash(cur ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
                const int cn = n0 + wn + 16 * j + (lane & 15);
                if (row >= g.M || cn >= g.N) continue;
                const float v = acc[i][j][r];
                const int64_t o = (int64_t)row * g.ldc + cn;
                if (EPI == EPI_SILU) {
                    const float z = v + g.bias[cn];
                    if (g.zout) g.zout[o] = z;
                    g.C[o] = z * logistic(z);
                } else {
                    float z = v + (g.bias ? g.bias[cn] : 0.f);
                    if (g.mu) z = g.mu[cn] + g.sd[cn] * z;
                    g.C[o] = z;
                }
            }
}

// Inference through every layer in one kernel: a block takes 64 rows, keeps
// their activations in LDS as BF16 (two 64 x 256 buffers), and each wave
// computes 64 output columns of a layer (4 x 4 MFMA tiles), its weight
// fragments read from L2 one k-step ahead.  Widths <= 256; the input width and
// every hidden width a multiple of 32.
constexpr int FMB = 64, FMW = 256, FALD = FMW + 8;

struct FusedArgs {
    const float* in;
    int64_t B;
    float* out;
    int L;
    int dims[LABFM_MLP_MAX_LAYERS + 1];
    const __bf16* W[LABFM_MLP_MAX_LAYERS];
    const float* b[LABFM_MLP_MAX_LAYERS];
    const float* mu;
    const float* sd;
};

__global__ __launch_bounds__(256) void k_mlp_fused(FusedArgs f) {
    __shared__ __bf16 act[2][FMB][FALD];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * FMB;
    const int K0 = f.dims[0];
    for (int e = tid * 4; e < FMB * K0; e += 256 * 4) {  // K0 % 4 == 0: a float4 never straddles rows
        const int r = e / K0, k = e % K0;
        floatx4 v = floatx4{0.f, 0.f, 0.f, 0.f};
        if (r0 + r < f.B) v = *(const floatx4*)(f.in + (r0 + r) * K0 + k);
#pragma unroll
        for (int q = 0; q < 4; ++q) act[0][r][k + q] = (__bf16)v[q];
    }
    __syncthreads();
    int cur = 0;
    for (int l = 0; l < f.L; ++l) {
        const int K = f.dims[l], N = f.dims[l + 1];
        const __bf16* W = f.W[l];
        const int wn = 64 * w;
        floatx4 acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
        if (wn < N) {  // wave-uniform
            bf16x8 bf[4], bn[4];
            auto wload = [&](int k0, bf16x8(&dst)[4]) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int n = wn + 16 * j + (lane & 15);
                    if (n < N) {
                        dst[j] = *(const bf16x8*)(W + (int64_t)n * K + k0 + 8 * (lane >> 4));
                    } else {
#pragma unroll
                        for (int e = 0; e < 8; ++e) dst[j][e] = (__bf16)0.f;
                    }
                }
            };
            wload(0, bf);
            for (int k0 = 0; k0 < K; k0 += 32) {
                if (k0 + 32 < K) wload(k0 + 32, bn);
                bf16x8 af[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) af[i] = *(const bf16x8*)&act[cur][16 * i + (lane & 15)][k0 + 8 * (lane >> 4)];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
#pragma unroll
                for (int j = 0; j < 4; ++j) bf[j] = bn[j];
            }
        }
        const bool last = l + 1 == f.L;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * i + 4 * (lane >> 4) + r;
                    const int cn = wn + 16 * j + (lane & 15);
                    if (cn >= N) continue;
                    const float z = acc[i][j][r] + f.b[l][cn];
                    if (!last) {
                        act[cur ^ 1][row][cn] = (__bf16)(z * logistic(z));
                    } else if (r0 + row < f.B) {
                        f.out[(r0 + row) * N + cn] = f.mu ? f.mu[cn] + f.sd[cn] * z : z;
                    }
                }
        __syncthreads();
        cur ^= 1;
    }
}

bool fused_ok(const labfm_mlp* net, const float* in) {
    const int L = net->n_layers;
    if (net->dims[0] % 32 != 0 || net->dims[0] > FMW || ((uintptr_t)in & 15) != 0) return false;
    for (int l = 1; l <= L; ++l) {
        if (net->dims[l] > FMW) return false;
        if (l < L && net->dims[l] % 32 != 0) return false;
    }
    for (int l = 0; l < L; ++l)
        if (((uintptr_t)net->W[l] & 15) != 0) return false;
    return true;
}

// forward layer: the tiled kernel when K and the row strides allow 16-byte loads
// forward layer: the tiled kernel when K and the row strides allow 16-byte loads
template <int EPI>
void gemm_forward(const GemmArgs& g, hipStream_t st) {
    const bool fast = g.K % FBK == 0 && g.lak == 1 && g.lbk == 1 && g.lam % 4 == 0 && g.lbn % 8 == 0 &&
                      ((uintptr_t)g.A & 15) == 0 && ((uintptr_t)g.B & 15) == 0;
    if (fast) {
        const dim3 grid((unsigned)((g.N + FBN - 1) / FBN), (unsigned)((g.M + FBM - 1) / FBM));
        k_gemm_fwd<EPI><<<grid, 256, 0, st>>>(g);
    } else {
        const dim3 grid((unsigned)((g.N + GBN - 1) / GBN), (unsigned)((g.M + GBM - 1) / GBM));
        k_gemm<__bf16, true, true, EPI><<<grid, 256, 0, st>>>(g);
    }
}

template <typename TB, bool AK, bool BK, int EPI>
void gemm(const GemmArgs& g, hipStream_t st) {
    const dim3 grid((unsigned)((g.N + GBN - 1) / GBN), (unsigned)((g.M + GBM - 1) / GBM));
    k_gemm<TB, AK, BK, EPI><<<grid, 256, 0, st>>>(g);
}

// ------------------------------------------------------------------ column sums (bias gradients)

constexpr int CS_SLICES = 64;

// partial[s][n] = sum of rows [s*rps, (s+1)*rps) of column n; 64 columns x 4 row lanes per block
__global__ __launch_bounds__(256) void k_colsum_partial(const float* __restrict__ Z, int64_t M, int N, int64_t ld,
                                                        int64_t rps, float* __restrict__ partial) {
    __shared__ float red[4][64];
    const int c = threadIdx.x & 63, r = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + c;
    const int64_t r0 = (int64_t)blockIdx.y * rps;
    const int64_t r1 = r0 + rps < M ? r0 + rps : M;
    float s = 0.f;
    if (n < N)
        for (int64_t m = r0 + r; m < r1; m += 4) s += Z[m * ld + n];
    red[r][c] = s;
    __syncthreads();
    if (r == 0 && n < N) partial[(int64_t)blockIdx.y * N + n] = red[0][c] + red[1][c] + red[2][c] + red[3][c];
}

__global__ void k_colsum_final(const float* __restrict__ partial, int slices, int N, float* __restrict__ out) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int k = 0; k < slices; ++k) s += partial[(int64_t)k * N + n];
    out[n] = s;
}

// ------------------------------------------------------------------ moment-residual loss

// Per sample s (one wavefront): Psi^d = mu + sd * y^d, r^d = M_s Psi^d - C^d,
// loss[s] = sum_d |r^d|^2, dy^d = 2 sd * (M_s^T r^d) / B.  M_s [p][p], row = monomial.
__global__ __launch_bounds__(64) void k_moment_loss(const float* __restrict__ y, const float* __restrict__ M,
                                                    const float* __restrict__ mu, const float* __restrict__ sd,
                                                    OpList ops, int P, int64_t B, float* __restrict__ dy,
                                                    double* __restrict__ loss) {
    __shared__ double sPsi[MAXOPS][64];
    __shared__ double sR[MAXOPS][64];
    const int lane = threadIdx.x;
    const int nops = ops.nops;
    const int ld = nops * P;
    for (int64_t s = blockIdx.x; s < B; s += gridDim.x) {
        const float* Ms = M + s * (int64_t)P * P;
        if (lane < P)
            for (int d = 0; d < nops; ++d)
                sPsi[d][lane] = (double)mu[d * P + lane] + (double)sd[d * P + lane] * (double)y[s * ld + d * P + lane];
        __syncthreads();
        double l2 = 0.0;
        if (lane < P) {
            for (int d = 0; d < nops; ++d) {
                double acc = 0.0;
                for (int q = 0; q < P; ++q) acc = fma((double)Ms[lane * P + q], sPsi[d][q], acc);
                const double r = acc - target(ops.op[d], lane);
                sR[d][lane] = r;
                l2 = fma(r, r, l2);
            }
        }
        for (int off = 32; off >= 1; off >>= 1) l2 += __shfl_xor(l2, off, 64);
        if (lane == 0) loss[s] = l2;
        __syncthreads();
        if (lane < P) {
            for (int d = 0; d < nops; ++d) {
                double acc = 0.0;
                for (int m = 0; m < P; ++m) acc = fma((double)Ms[m * P + lane], sR[d][m], acc);
                dy[s * ld + d * P + lane] = (float)(2.0 * (double)sd[d * P + lane] * acc / (double)B);
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ Adam, cast

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, __bf16* __restrict__ pb, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    p[i] = pi;
    if (pb) pb[i] = (__bf16)pi;
}

__global__ void k_cast_bf16(const float* __restrict__ src, __bf16* __restrict__ dst, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (__bf16)src[i];
}

inline unsigned blocks1d(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

int maxdim(const labfm_mlp* net) {
    int m = 0;
    for (int l = 0; l <= net->n_layers; ++l) m = net->dims[l] > m ? net->dims[l] : m;
    return m;
}

labfm_err colsum(Context* c, const float* Z, int64_t M, int N, int64_t ld, float* out, hipStream_t st) {
    const int slices = (int)(M < CS_SLICES ? (M > 0 ? M : 1) : CS_SLICES);
    const int64_t rps = (M + slices - 1) / slices;
    labfm_err e = ensure(c->mlp_part, sizeof(float) * (size_t)slices * N);
    if (e != LABFM_OK) return e;
    float* part = (float*)c->mlp_part.p;
    k_colsum_partial<<<dim3(blocks1d(N, 64), slices), 256, 0, st>>>(Z, M, N, ld, rps, part);
    k_colsum_final<<<blocks1d(N, 256), 256, 0, st>>>(part, slices, N, out);
    return LABFM_OK;
}

// ------------------------------------------------------------------ training data
// For every node (all of order K) the moment matrix M = sum_j X(d_j) W(d_j)^T
// of eq. (disc_form) in scaled offsets, written in FP32 [p][p] (row =
// monomial) as assembled, and the coefficients Psi^d of eq. (lsys) from the
// FP64 path's equilibration, partial-pivot LU and one solve (no refinement),
// in FP32, operator-major [nops][p].  Nodes that are not OK get zeros.  The
// assembly, equilibration and LU are the FP64 weight kernel's steps.
template <int K, int FAM>
__global__ __launch_bounds__(64) void k_moment_systems(WeightArgs a, OpList ops, float* __restrict__ Mo,
                                                       float* __restrict__ psio, int8_t* __restrict__ sto) {
    constexpr int P = p_of_k(K);
    constexpr int BS = (P + 7) / 8;
    constexpr int PP = 8 * BS;
    constexpr int LD = P + 1;

    __shared__ double sM[P * LD];
    __shared__ double sChunk[2 * CH * PP];
    __shared__ double sD[2][NMAX];
    __shared__ double sRs[P], sCs[P];
    __shared__ int sPerm[P];

    const NodeSet& S = a.one;
    const int lane = threadIdx.x;
    const int nops = ops.nops;

    for (int64_t i = blockIdx.x; i < S.n; i += gridDim.x) {
        const int64_t s0 = S.row_ptr[i];
        const int N = (int)(S.row_ptr[i + 1] - s0);
        const double h = 0.5 * S.R[i];
        int status = LABFM_ST_OK;
        for (int d = 0; d < nops; ++d)
            if (K < min_order(ops.op[d])) status = LABFM_ST_ORDER_TOO_LOW;
        if (status == LABFM_ST_OK && N < P) status = LABFM_ST_TOO_FEW;
        if (status == LABFM_ST_OK && N > NMAX) status = LABFM_ST_TOO_MANY;
        if (status == LABFM_ST_OK) {
            const double xi = S.x[i], yi = S.y[i];
            bool bad = false;
            for (int q = lane; q < N; q += 64) {
                const int32_t j = S.col[s0 + q];
                const double dx = min_image(S.x[j] - xi, S.Lx, S.perx) / h;
                const double dy = min_image(S.y[j] - yi, S.Ly, S.pery) / h;
                sD[0][q] = dx;
                sD[1][q] = dy;
                if (FAM != LABFM_ABF_HERMITE && dx == 0.0 && dy == 0.0) bad = true;
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

            // the moment matrix as assembled, before any scaling
            for (int e = lane; e < P * P; e += 64) Mo[i * (int64_t)(P * P) + e] = (float)sM[(e / P) * LD + e % P];
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
                double b[MAXOPS];
#pragma unroll
                for (int d = 0; d < MAXOPS; ++d) b[d] = (d < nops) ? target(ops.op[d], lane) : 0.0;
                lu_solve<P, LD>(sM, sRs, sCs, sPerm, b, nops);
                if (lane < P)
                    for (int d = 0; d < nops; ++d) psio[(i * nops + d) * (int64_t)P + lane] = (float)b[d];
            }
        }
        if (status != LABFM_ST_OK) {
            for (int e = lane; e < P * P; e += 64) Mo[i * (int64_t)(P * P) + e] = 0.f;
            for (int e = lane; e < nops * P; e += 64) psio[i * (int64_t)(nops * P) + e] = 0.f;
        }
        if (lane == 0) sto[i] = (int8_t)status;
        __syncthreads();
    }
}

template <int K, int FAM>
void launch_moment_systems(const WeightArgs& a, const OpList& ops, float* Mo, float* psio, int8_t* sto,
                           hipStream_t st) {
    static int grid = 0;
    if (grid == 0) {
        int dev = 0, ncu = 0, per = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_moment_systems<K, FAM>, 64, 0);
        grid = (ncu > 0 ? ncu : 256) * (per > 0 ? per : 1);
    }
    k_moment_systems<K, FAM><<<grid, 64, 0, st>>>(a, ops, Mo, psio, sto);
}

template <int FAM>
void moment_systems_fam(const WeightArgs& a, const OpList& ops, int k, float* Mo, float* psio, int8_t* sto,
                        hipStream_t st) {
    switch (k) {
        case 1: launch_moment_systems<1, FAM>(a, ops, Mo, psio, sto, st); break;
        case 2: launch_moment_systems<2, FAM>(a, ops, Mo, psio, sto, st); break;
        case 3: launch_moment_systems<3, FAM>(a, ops, Mo, psio, sto, st); break;
        case 4: launch_moment_systems<4, FAM>(a, ops, Mo, psio, sto, st); break;
        case 5: launch_moment_systems<5, FAM>(a, ops, Mo, psio, sto, st); break;
        case 6: launch_moment_systems<6, FAM>(a, ops, Mo, psio, sto, st); break;
        case 7: launch_moment_systems<7, FAM>(a, ops, Mo, psio, sto, st); break;
        default: launch_moment_systems<8, FAM>(a, ops, Mo, psio, sto, st); break;
    }
}

}  // namespace

// ------------------------------------------------------------------ host entry points (internal)

labfm_err mlp_features(Context* c, const double* x, const double* y, const double* R, const int64_t* row_ptr,
                       const int32_t* col, int64_t first, int64_t count, double Lx, double Ly, int perx, int pery,
                       int kmax, float* feat, hipStream_t st) {
    if (count <= 0) return LABFM_OK;
    KernelTimer timer(c, "mlp_features", st);
    const unsigned grid = (unsigned)(count < 65536 ? count : 65536);
    k_features<<<grid, 64, 0, st>>>(x, y, R, row_ptr, col, first, count, Lx, Ly, perx, pery, kmax, feat);
    LABFM_HIP_CHECK(hipGetLastError());
    return LABFM_OK;
}

size_t mlp_cache_floats(const labfm_mlp* net, int64_t B) {
    size_t s = 0;
    for (int l = 0; l + 1 < net->n_layers; ++l) s += 2 * (size_t)B * net->dims[l + 1];
    return s;
}

labfm_err mlp_forward(Context* c, const labfm_mlp* net, const float* in, int64_t B, float* out, float* cache,
                      int denorm, hipStream_t st) {
    if (B <= 0) return LABFM_OK;
    const int L = net->n_layers;
    if (!cache && fused_ok(net, in)) {
        KernelTimer timer(c, "mlp_forward", st);
        FusedArgs f{};
        f.in = in;
        f.B = B;
        f.out = out;
        f.L = L;
        for (int l = 0; l <= L; ++l) f.dims[l] = net->dims[l];
        for (int l = 0; l < L; ++l) {
            f.W[l] = (const __bf16*)net->W[l];
            f.b[l] = net->b[l];
        }
        f.mu = denorm ? net->mu : nullptr;
        f.sd = denorm ? net->sd : nullptr;
        k_mlp_fused<<<(unsigned)((B + FMB - 1) / FMB), 256, 0, st>>>(f);
        LABFM_HIP_CHECK(hipGetLastError());
        return LABFM_OK;
    }
    float* ping = nullptr;
    float* pong = nullptr;
    if (!cache && L > 1) {
        const size_t per = (size_t)B * maxdim(net);
        labfm_err e = ensure(c->mlp_act, sizeof(float) * 2 * per);
        if (e != LABFM_OK) return e;
        ping = (float*)c->mlp_act.p;
        pong = ping + per;
    }
    KernelTimer timer(c, "mlp_forward", st);
    const float* H = in;
    size_t off = 0;
    for (int l = 0; l < L; ++l) {
        const int kin = net->dims[l], nout = net->dims[l + 1];
        GemmArgs g{};
        g.M = (int)B;
        g.N = nout;
        g.K = kin;
        g.A = H;
        g.lam = kin;
        g.lak = 1;
        g.B = net->W[l];
        g.lbk = 1;
        g.lbn = kin;
        g.ldc = nout;
        g.bias = net->b[l];
        if (l + 1 < L) {
            if (cache) {
                g.zout = cache + off;
                g.C = cache + off + (size_t)B * nout;
                off += 2 * (size_t)B * nout;
            } else {
                g.C = (l % 2 == 0) ? ping : pong;
            }
            gemm_forward<EPI_SILU>(g, st);
        } else {
            g.C = out;
            if (denorm) {
                g.mu = net->mu;
                g.sd = net->sd;
            }
            gemm_forward<EPI_LINEAR>(g, st);
        }
        H = g.C;
    }
    LABFM_HIP_CHECK(hipGetLastError());
    return LABFM_OK;
}

labfm_err mlp_backward(Context* c, const labfm_mlp* net, const float* in, const float* cache, const float* dout,
                       int64_t B, const labfm_mlp_grads* gr, hipStream_t st) {
    if (B <= 0) return LABFM_OK;
    const int L = net->n_layers;
    const size_t per = (size_t)B * maxdim(net);
    labfm_err e = ensure(c->mlp_act, sizeof(float) * 2 * per);
    if (e != LABFM_OK) return e;
    float* buf[2] = {(float*)c->mlp_act.p, (float*)c->mlp_act.p + per};
    // offsets of (Z_l, H_l) of the hidden layers in the cache
    size_t zoff[LABFM_MLP_MAX_LAYERS], hoff[LABFM_MLP_MAX_LAYERS];
    size_t off = 0;
    for (int l = 0; l + 1 < L; ++l) {
        zoff[l] = off;
        hoff[l] = off + (size_t)B * net->dims[l + 1];
        off += 2 * (size_t)B * net->dims[l + 1];
    }
    KernelTimer timer(c, "mlp_backward", st);
    const float* dZ = dout;
    for (int l = L - 1; l >= 0; --l) {
        const int nin = net->dims[l], nout = net->dims[l + 1];
        const float* Hin = l == 0 ? in : cache + hoff[l - 1];
        // dW_l = dZ^T Hin  ([nout][nin], reduction over the batch)
        GemmArgs g{};
        g.M = nout;
        g.N = nin;
        g.K = (int)B;
        g.A = dZ;
        g.lam = 1;
        g.lak = nout;
        g.B = Hin;
        g.lbk = nin;
        g.lbn = 1;
        g.C = gr->W[l];
        g.ldc = nin;
        gemm<float, false, false, EPI_PLAIN>(g, st);
        if ((e = colsum(c, dZ, B, nout, nout, gr->b[l], st)) != LABFM_OK) return e;
        if (l > 0) {
            // dZ_{l-1} = (dZ W_l) * silu'(Z_{l-1})
            GemmArgs h{};
            h.M = (int)B;
            h.N = nin;
            h.K = nout;
            h.A = dZ;
            h.lam = nout;
            h.lak = 1;
            h.B = net->W[l];
            h.lbk = nin;
            h.lbn = 1;
            float* next = buf[l % 2];
            h.C = next;
            h.ldc = nin;
            h.zin = cache + zoff[l - 1];
            gemm<__bf16, true, false, EPI_DSILU>(h, st);
            dZ = next;
        }
    }
    LABFM_HIP_CHECK(hipGetLastError());
    return LABFM_OK;
}

labfm_err mlp_moment_loss(Context* c, const float* y, const float* M, const float* mu, const float* sd, int order,
                          unsigned opbits, int64_t B, float* dy, double* loss, hipStream_t st) {
    if (B <= 0) return LABFM_OK;
    OpList ops{};
    for (int b = 0; b < 5; ++b)
        if (opbits & (1u << b)) ops.op[ops.nops++] = 1u << b;
    const int P = (order * order + 3 * order) / 2;
    KernelTimer timer(c, "mlp_loss", st);
    const unsigned grid = (unsigned)(B < 65536 ? B : 65536);
    k_moment_loss<<<grid, 64, 0, st>>>(y, M, mu, sd, ops, P, B, dy, loss);
    LABFM_HIP_CHECK(hipGetLastError());
    return LABFM_OK;
}

labfm_err mlp_adam(Context* c, float* p, const float* g, float* m, float* v, void* pb, int64_t n, const labfm_adam* hp,
                   int64_t t, hipStream_t st) {
    if (n <= 0) return LABFM_OK;
    const double c1 = 1.0 / (1.0 - std::pow((double)hp->beta1, (double)t));
    const double c2 = 1.0 / (1.0 - std::pow((double)hp->beta2, (double)t));
    KernelTimer timer(c, "mlp_adam", st);
    k_adam<<<blocks1d(n, 256), 256, 0, st>>>(p, g, m, v, (__bf16*)pb, n, (float)hp->lr, (float)hp->beta1,
                                             (float)hp->beta2, (float)hp->eps, (float)c1, (float)c2);
    LABFM_HIP_CHECK(hipGetLastError());
    return LABFM_OK;
}

labfm_err mlp_cast_bf16(const float* src, void* dst, int64_t n, hipStream_t st) {
    if (n <= 0) return LABFM_OK;
    k_cast_bf16<<<blocks1d(n, 256), 256, 0, st>>>(src, (__bf16*)dst, n);
    LABFM_HIP_CHECK(hipGetLastError());
    return LABFM_OK;
}

// Warm-started weights: features and network output for every node (chunks of
// MLP_CHUNK nodes), then the mixed kernels start the order-net->order systems
// from Psi0 and the FP64 kernels take the nodes that do not converge.
constexpr int64_t MLP_CHUNK = 65536;

labfm_err moment_systems(Context* c, const WeightArgs& a, int k, float* M, float* psi, int8_t* status,
                         hipStream_t st) {
    if (a.one.n == 0) return LABFM_OK;
    OpList ops{};
    ops.nops = 0;
    for (int b = 0; b < 5; ++b)
        if (a.ops & (1u << b)) ops.op[ops.nops++] = 1u << b;
    KernelTimer timer(c, "moment_systems", st);
    if (a.abf == LABFM_ABF_HERMITE)
        moment_systems_fam<LABFM_ABF_HERMITE>(a, ops, k, M, psi, status, st);
    else if (a.abf == LABFM_ABF_PAPER)
        moment_systems_fam<LABFM_ABF_PAPER>(a, ops, k, M, psi, status, st);
    else
        moment_systems_fam<LABFM_ABF_PAPER_D1>(a, ops, k, M, psi, status, st);
    LABFM_HIP_CHECK(hipGetLastError());
    return LABFM_OK;
}

labfm_err weights_mlp(Context* c, const WeightArgs& a0, int32_t* wl, int32_t* rl, const labfm_mlp* net,
                      hipStream_t st, bool direct) {
    const NodeSet& S = a0.one;
    const int64_t n = S.n;
    const int L = net->n_layers;
    const int nout = net->dims[L];
    labfm_err e = ensure(c->mlp_psi, sizeof(float) * (size_t)n * nout);
    if (e != LABFM_OK) return e;
    float* psi0 = (float*)c->mlp_psi.p;
    const int64_t ch = n < MLP_CHUNK ? n : MLP_CHUNK;
    if ((e = ensure(c->mlp_feat, sizeof(float) * (size_t)ch * net->dims[0])) != LABFM_OK) return e;
    float* feat = (float*)c->mlp_feat.p;
    for (int64_t f = 0; f < n; f += ch) {
        const int64_t cnt = n - f < ch ? n - f : ch;
        if ((e = mlp_features(c, S.x, S.y, S.R, S.row_ptr, S.col, f, cnt, S.Lx, S.Ly, S.perx, S.pery, net->kmax, feat,
                              st)) != LABFM_OK)
            return e;
        if ((e = mlp_forward(c, net, feat, cnt, psi0 + f * nout, nullptr, 1, st)) != LABFM_OK) return e;
    }
    WeightArgs a = a0;
    a.one.psi0 = psi0;
    a.psi0_order = net->order;
    a.psi0_ld = nout;
    return weights_mixed(c, a, &a.one, wl, rl, 0u, st, direct ? net->order : 0, &c->factors);
}

}  // namespace labfm
