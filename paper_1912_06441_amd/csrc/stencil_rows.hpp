// stencil_rows.hpp -- row-parallel stencil sums shared by the application,
// RK4 and Burgers kernels: L^d_i(x) = sum_{q in row i} w_d[q] (x[col[q]] - x_i)
// (Sec. 2 eq. general_do), G lanes per CSR row, U loads in flight per lane.
#pragma once

#include "labfm_internal.hpp"

namespace labfm {
namespace rows {

// Lanes per row (G) and loads in flight per lane (U): G*U entries of a row
// are requested before the first gather result is used.  Swept on the
// 512x512 (N~60) and 1024x1024 (N~49) neighbour structures: FP64 streams
// favour G=16, U=4; FP32 streams G=8, U=8.
template <typename T>
struct Shape;
template <>
struct Shape<double> {
    static constexpr int G = 16, U = 4;
};
template <>
struct Shape<float> {
    static constexpr int G = 8, U = 8;
};

template <typename T, int G>
__device__ inline T group_sum(T v) {
#pragma unroll
    for (int off = G / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, G);
    return v;
}

// NW weight streams over one CSR row, lane `sub` of G:
//   acc[d] += sum_{q in row, q = sub mod G} w_d[q] (x[col[q]] - xi).
// Every index and weight load of a U-block is issued before its gathers.
template <typename T, int NW>
struct WPtrs {
    const T* p[NW];
};

template <typename T, int G, int U, int NW>
__device__ inline void row_sums(const int32_t* __restrict__ col, int64_t s, int64_t e, int sub, const WPtrs<T, NW>& w,
                                const T* __restrict__ x, T xi, T (&acc)[NW]) {
    for (int64_t q0 = s + sub; q0 < e; q0 += (int64_t)G * U) {
        int c[U];
        T wv[U][NW];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int64_t q = q0 + (int64_t)k * G;
            c[k] = q < e ? col[q] : -1;
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int64_t q = q0 + (int64_t)k * G;
#pragma unroll
            for (int d = 0; d < NW; ++d) wv[k][d] = q < e ? w.p[d][q] : T(0);
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const T dx = c[k] >= 0 ? x[c[k]] - xi : T(0);
#pragma unroll
            for (int d = 0; d < NW; ++d) acc[d] += wv[k][d] * dx;
        }
    }
}

// The same sums for two fields x and y over one read of the index and weight
// streams: ax[d] += w_d (x_j - x_i), ay[d] += w_d (y_j - y_i).
template <typename T, int G, int U, int NW>
__device__ inline void row_sums2(const int32_t* __restrict__ col, int64_t s, int64_t e, int sub,
                                 const WPtrs<T, NW>& w, const T* __restrict__ x, const T* __restrict__ y, T xi,
                                 T yi, T (&ax)[NW], T (&ay)[NW]) {
    for (int64_t q0 = s + sub; q0 < e; q0 += (int64_t)G * U) {
        int c[U];
        T wv[U][NW];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int64_t q = q0 + (int64_t)k * G;
            c[k] = q < e ? col[q] : -1;
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int64_t q = q0 + (int64_t)k * G;
#pragma unroll
            for (int d = 0; d < NW; ++d) wv[k][d] = q < e ? w.p[d][q] : T(0);
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const T dx = c[k] >= 0 ? x[c[k]] - xi : T(0);
            const T dy = c[k] >= 0 ? y[c[k]] - yi : T(0);
#pragma unroll
            for (int d = 0; d < NW; ++d) {
                ax[d] += wv[k][d] * dx;
                ay[d] += wv[k][d] * dy;
            }
        }
    }
}

// stage update: k is the stage derivative at node i; on Dirichlet nodes it is
// kfix[i] when an imposed derivative is given, else zero
template <typename T>
__device__ inline void rk4_update(int stage, T k, T dt, int64_t i, const int8_t* fixed, T* u, T* acc, T* us_out,
                                  const T* kfix = nullptr) {
    if (fixed && fixed[i]) k = kfix ? kfix[i] : T(0);
    const T ui = u[i];
    if (stage == 0) {
        acc[i] = k;
        us_out[i] = ui + T(0.5) * dt * k;
    } else if (stage == 1) {
        acc[i] = acc[i] + T(2) * k;
        us_out[i] = ui + T(0.5) * dt * k;
    } else if (stage == 2) {
        acc[i] = acc[i] + T(2) * k;
        us_out[i] = ui + dt * k;
    } else {
        u[i] = ui + dt / T(6) * (acc[i] + k);
    }
}

template <typename T>
inline unsigned blocks_for(int64_t n) {
    return (unsigned)((n * Shape<T>::G + 255) / 256);
}

}  // namespace rows
}  // namespace labfm
