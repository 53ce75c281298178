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

// Two components stored as one pair per node, so that a row gathers both
// with a single load per entry.
template <typename T>
struct Vec2;
template <>
struct Vec2<float> {
    using type = float2;
};
template <>
struct Vec2<double> {
    using type = double2;
};

// The same sums for two fields held as pairs, over one read of the index and
// weight streams: ax[d] += w_d (xy_j.x - x_i), ay[d] += w_d (xy_j.y - y_i).
template <typename T, int G, int U, int NW>
__device__ inline void row_sums2p(const int32_t* __restrict__ col, int64_t s, int64_t e, int sub,
                                  const WPtrs<T, NW>& w, const typename Vec2<T>::type* __restrict__ xy, T xi, T yi,
                                  T (&ax)[NW], T (&ay)[NW]) {
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
            T dx = T(0), dy = T(0);
            if (c[k] >= 0) {
                const typename Vec2<T>::type g = xy[c[k]];
                dx = g.x - xi;
                dy = g.y - yi;
            }
#pragma unroll
            for (int d = 0; d < NW; ++d) {
                ax[d] += wv[k][d] * dx;
                ay[d] += wv[k][d] * dy;
            }
        }
    }
}

// Classical RK4 stage update of one node (Sec. 5.1).  The node's own values
// are read by rk4_load before the row sums, so that these loads overlap the
// stencil gathers rather than following the group reduction; rk4_store then
// applies the stage with the derivative k.  On Dirichlet nodes k is replaced
// by the imposed derivative kfix[i] when one is given, else by zero.
template <typename T>
struct Rk4Node {
    T u, acc, kfix;
    bool fix;
};

template <typename T>
__device__ inline Rk4Node<T> rk4_load(int stage, int64_t i, const int8_t* fixed, const T* u, const T* acc,
                                      const T* kfix = nullptr) {
    Rk4Node<T> s;
    s.fix = fixed && fixed[i];
    s.kfix = (s.fix && kfix) ? kfix[i] : T(0);
    s.u = u[i];
    s.acc = stage > 0 ? acc[i] : T(0);
    return s;
}

// applies the stage and returns the next stage state (stages 0-2); the last
// stage writes the new value to u[i] and returns zero
template <typename T>
__device__ inline T rk4_stage(int stage, T k, T dt, int64_t i, const Rk4Node<T>& s, T* u, T* acc) {
    if (s.fix) k = s.kfix;
    if (stage == 0) {
        acc[i] = k;
        return s.u + T(0.5) * dt * k;
    }
    if (stage == 1) {
        acc[i] = s.acc + T(2) * k;
        return s.u + T(0.5) * dt * k;
    }
    if (stage == 2) {
        acc[i] = s.acc + T(2) * k;
        return s.u + dt * k;
    }
    u[i] = s.u + dt / T(6) * (s.acc + k);
    return T(0);
}

template <typename T>
__device__ inline void rk4_store(int stage, T k, T dt, int64_t i, const Rk4Node<T>& s, T* u, T* acc, T* us_out) {
    const T us = rk4_stage<T>(stage, k, dt, i, s, u, acc);
    if (stage < 3) us_out[i] = us;
}

template <typename T>
inline unsigned blocks_for(int64_t n) {
    return (unsigned)((n * Shape<T>::G + 255) / 256);
}

}  // namespace rows
}  // namespace labfm
