// weights_common.hpp -- helpers shared by the FP64 and mixed-precision weight kernels.
#pragma once

#include "labfm_internal.hpp"
#include "basis.hpp"

namespace labfm {
namespace wk {

constexpr int CH = 16;  // neighbours per basis chunk
constexpr int cmax(int a, int b) { return a > b ? a : b; }

__device__ inline double bcast(double v, int src) {
    int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

__device__ inline double wave_max(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ inline double wave_max_double(double v) { return wave_max(v); }
__device__ inline float wave_max_float(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ inline double min_image(double d, double L, int per) {
    if (!per) return d;
    if (d > 0.5 * L) return d - L;
    if (d < -0.5 * L) return d + L;
    return d;
}

// target vector element m of operator code op (bit value); l = derivative order
__device__ inline double target(unsigned op, int m) {
    switch (op) {
        case LABFM_OP_DX: return m == 0 ? 1.0 : 0.0;
        case LABFM_OP_DY: return m == 1 ? 1.0 : 0.0;
        case LABFM_OP_LAP: return (m == 2 || m == 4) ? 1.0 : 0.0;
        case LABFM_OP_BIHARM: return m == 9 ? -1.0 : (m == 11 ? -2.0 : (m == 13 ? -1.0 : 0.0));
        case LABFM_OP_TRIHARM:
            return m == 20 ? 1.0 : (m == 22 ? 3.0 : (m == 24 ? 3.0 : (m == 26 ? 1.0 : 0.0)));
    }
    return 0.0;
}
__host__ __device__ inline int deriv_order(unsigned op) {
    return op == LABFM_OP_DX || op == LABFM_OP_DY ? 1 : (op == LABFM_OP_LAP ? 2 : (op == LABFM_OP_BIHARM ? 4 : 6));
}
__host__ __device__ inline int min_order(unsigned op) {
    return op == LABFM_OP_BIHARM ? 4 : (op == LABFM_OP_TRIHARM ? 6 : (op == LABFM_OP_LAP ? 2 : 1));
}

struct OpList {
    unsigned op[MAXOPS];
    int nops;
};


// Solve M z = b with the equilibrated, pivoted LU in LDS.  Lane m holds
// b[d] for original row m on entry; lane c holds z[d] for unknown c on exit.
template <int P, int LD, typename T>
__device__ inline void lu_solve(const T* sM, const T* sRs, const T* sCs, const int* sPerm, double (&b)[MAXOPS],
                                int nops) {
    const int lane = threadIdx.x;
    const int pr = lane < P ? sPerm[lane] : 0;
    const double rs = lane < P ? sRs[lane] : 0.0;
    double t[MAXOPS];
#pragma unroll
    for (int d = 0; d < MAXOPS; ++d) {
        double v = b[d] * rs;
        t[d] = __shfl(v, pr, 64);
    }
    // forward: unit lower triangle (factor entries loaded four steps ahead)
    int c = 0;
    for (; c + 4 <= P - 1; c += 4) {
        double l[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) l[q] = (lane > c + q && lane < P) ? (double)sM[lane * LD + c + q] : 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int d = 0; d < MAXOPS; ++d)
                if (d < nops) t[d] -= l[q] * bcast(t[d], c + q);
    }
    for (; c < P - 1; ++c) {
        const double l = (lane > c && lane < P) ? (double)sM[lane * LD + c] : 0.0;
#pragma unroll
        for (int d = 0; d < MAXOPS; ++d)
            if (d < nops) t[d] -= l * bcast(t[d], c);
    }
    // backward
    c = P - 1;
    for (; c - 3 >= 0; c -= 4) {
        double dg[4], u[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            dg[q] = (double)sM[(c - q) * LD + c - q];
            u[q] = (lane < c - q) ? (double)sM[lane * LD + c - q] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int d = 0; d < MAXOPS; ++d) {
                if (d < nops) {
                    if (lane == c - q) t[d] = t[d] / dg[q];
                    t[d] -= u[q] * bcast(t[d], c - q);
                }
            }
    }
    for (; c >= 0; --c) {
        const double diag = (double)sM[c * LD + c];
        const double u = (lane < c) ? (double)sM[lane * LD + c] : 0.0;
#pragma unroll
        for (int d = 0; d < MAXOPS; ++d) {
            if (d < nops) {
                if (lane == c) t[d] = t[d] / diag;
                t[d] -= u * bcast(t[d], c);
            }
        }
    }
    const double cs = lane < P ? sCs[lane] : 0.0;
#pragma unroll
    for (int d = 0; d < MAXOPS; ++d) b[d] = t[d] * cs;
}

// Work item g -> (node set, node index within it).
__device__ inline void resolve(const WeightArgs& a, int64_t g, NodeSet& S, int64_t& i) {
    if (a.nsets <= 1) {
        S = a.one;
        i = g;
        return;
    }
    int lo = 0, hi = a.nsets - 1;  // largest s with set_off[s] <= g
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.set_off[mid] <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    S = a.sets[lo];
    i = g - a.set_off[lo];
}

}  // namespace wk
}  // namespace labfm
